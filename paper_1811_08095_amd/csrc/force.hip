// Fermion-force kernel: the link derivative of a hopping bilinear.
//
// For S = Re <chi, W psi> summed over the fifth dimension (W the hopping term
// of the 4D Wilson operator D_w that the optimal domain-wall operator applies
// on every slice; the HMC's fermion forces of §2 are sums of such terms with
// chi and psi built from the solutions of the normal equations), the only
// terms of S that contain the link U_mu(x) are
//     -1/2 b Re tr(U_mu(x) A) - 1/2 b Re tr(U_mu(x)^dag B),
//     A = sum_{s, spin} [(1 - gamma_mu) psi(x + mu, s)] (x) chi(x, s)^dag,
//     B = sum_{s, spin} [(1 + gamma_mu) psi(x, s)] (x) chi(x + mu, s)^dag,
// (b = bc_t on links that cross the t boundary), so S = Re tr(U_mu(x) M) + ...
// with M = -1/2 b (A + B^dag), and the force is F_mu(x) = TA(U_mu(x) M), the
// traceless anti-Hermitian part, for which dS/d eps = i tr(T F_mu(x)) when
// U_mu(x) -> exp(i eps T) U_mu(x).
//
// In the chiral basis sum_spin [(1 - s gamma) p] (x) c^dag = h_p (x) h_c^dag
// with h the same half-spinor projection of p and of c, so a lane forms each
// outer product from two 2 x 3 half spinors.  Thread layout as in the hopping
// kernel: a block holds 256 / Ns sites of one parity with Ns lanes each (s
// fastest); the lanes of a site add their 3 x 3 products over s through LDS in
// a fixed order (deterministic), then the site's lanes form the nine entries
// of TA(U M) and write (or add to) the canonical force field.  FP64 throughout.
#include "dev_common.h"
#include "kernels.h"

namespace odwf {

struct ForceArgs {
  const void* chi_own;   // chi on the sites of the output parity
  const void* psi_own;
  const void* chi_nb;    // chi on the opposite parity
  const void* psi_nb;
  const void* links;     // FP64 links of the output parity [h][8][18]
  cpx<double>* F;        // canonical [t][z][y][x][mu][3][3]
  int L[4];
  int h, Ns, par, bc_t, accumulate;
};

// partial[b][a] += sum_sigma hp[sigma][b] conj(hc[sigma][a])
__device__ __forceinline__ void outer_acc(const cpx<double> (&hp)[6], const cpx<double> (&hc)[6],
                                          cpx<double> (&m)[9]) {
#pragma unroll
  for (int b = 0; b < 3; b++)
#pragma unroll
    for (int a = 0; a < 3; a++) {
      cpx<double> v = m[b * 3 + a];
#pragma unroll
      for (int sg = 0; sg < 2; sg++) {
        const cpx<double> p = hp[sg * 3 + b], c = hc[sg * 3 + a];
        v.re += p.re * c.re + p.im * c.im;
        v.im += p.im * c.re - p.re * c.im;
      }
      m[b * 3 + a] = v;
    }
}

template <int MU>
__device__ __forceinline__ void link_products(const cpx<double> (&pn)[12], const cpx<double> (&cn)[12],
                                              const cpx<double> (&po)[12], const cpx<double> (&co)[12],
                                              cpx<double> (&A)[9], cpx<double> (&B)[9]) {
  cpx<double> hp[6], hc[6];
  project<MU, +1>(pn, hp);  // (1 - gamma_mu) psi(x + mu)
  project<MU, +1>(co, hc);  // with chi(x)
  outer_acc(hp, hc, A);
  project<MU, -1>(po, hp);  // (1 + gamma_mu) psi(x)
  project<MU, -1>(cn, hc);  // with chi(x + mu)
  outer_acc(hp, hc, B);
}

__global__ void __launch_bounds__(256) force_kernel(const ForceArgs a) {
  __shared__ double red[256 * 18];
  __shared__ double msum[64 * 18];
  const int Ns = a.Ns;
  const int spb = 256 / Ns;
  const int tid = threadIdx.x;
  const int sl = tid / Ns, s = tid - sl * Ns;
  const long j = (long)blockIdx.x * spb + sl;
  const bool valid = j < a.h;
  const int L0 = a.L[0], L1 = a.L[1], L2 = a.L[2], L3 = a.L[3];
  const int hx = L0 >> 1;
  int x = 0, y = 0, z = 0, t = 0;
  cpx<double> po[12], co[12];
  if (valid) {
    const int xh = (int)(j % hx);
    long rest = j / hx;
    y = (int)(rest % L1);
    rest /= L1;
    z = (int)(rest % L2);
    t = (int)(rest / L2);
    x = 2 * xh + ((y + z + t + a.par) & 1);
    load_site<SP64>(a.psi_own, nullptr, j, 0, s, 1, Ns, po);
    load_site<SP64>(a.chi_own, nullptr, j, 0, s, 1, Ns, co);
  }
#pragma unroll 1
  for (int mu = 0; mu < 4; mu++) {
    cpx<double> A[9], B[9];
#pragma unroll
    for (int k = 0; k < 9; k++) A[k] = B[k] = {0.0, 0.0};
    double bs = 1.0;
    if (valid) {
      int xx = x, yy = y, zz = z, tt = t;
      if (mu == 0) xx = x + 1 == L0 ? 0 : x + 1;
      if (mu == 1) yy = y + 1 == L1 ? 0 : y + 1;
      if (mu == 2) zz = z + 1 == L2 ? 0 : z + 1;
      if (mu == 3) {
        tt = t + 1 == L3 ? 0 : t + 1;
        if (t + 1 == L3 && a.bc_t < 0) bs = -1.0;
      }
      const long nj = (((long)tt * L2 + zz) * L1 + yy) * hx + (xx >> 1);
      cpx<double> pn[12], cn[12];
      load_site<SP64>(a.psi_nb, nullptr, nj, 0, s, 1, Ns, pn);
      load_site<SP64>(a.chi_nb, nullptr, nj, 0, s, 1, Ns, cn);
      switch (mu) {
        case 0: link_products<0>(pn, cn, po, co, A, B); break;
        case 1: link_products<1>(pn, cn, po, co, A, B); break;
        case 2: link_products<2>(pn, cn, po, co, A, B); break;
        default: link_products<3>(pn, cn, po, co, A, B); break;
      }
    }
    // this lane's share of M = -1/2 b (A + B^dag), then the sum over s
    __syncthreads();  // red and msum of the previous direction are consumed
#pragma unroll
    for (int b = 0; b < 3; b++)
#pragma unroll
      for (int c = 0; c < 3; c++) {
        const cpx<double> v = {-0.5 * bs * (A[b * 3 + c].re + B[c * 3 + b].re),
                               -0.5 * bs * (A[b * 3 + c].im - B[c * 3 + b].im)};
        red[tid * 18 + (b * 3 + c) * 2] = v.re;
        red[tid * 18 + (b * 3 + c) * 2 + 1] = v.im;
      }
    __syncthreads();
    for (int q = tid; q < spb * 18; q += blockDim.x) {
      const int site = q / 18, k = q - site * 18;
      double acc = 0.0;
      for (int u = 0; u < Ns; u++) acc += red[(site * Ns + u) * 18 + k];
      msum[q] = acc;
    }
    __syncthreads();
    // F = TA(U M): the Ns lanes of a site write entries e = s, s + Ns, ... < 9
    for (int e = s; valid && e < 9; e += Ns) {
      const int ra = e / 3, cb = e - ra * 3;
      const double* m = msum + sl * 18;
      const cpx<double>* U = reinterpret_cast<const cpx<double>*>(a.links) + (j * 8 + mu) * 9;
      auto X = [&](int r, int c) {  // (U M)[r][c]
        cpx<double> v = {0.0, 0.0};
#pragma unroll
        for (int k = 0; k < 3; k++) {
          const cpx<double> u = U[r * 3 + k], w = {m[(k * 3 + c) * 2], m[(k * 3 + c) * 2 + 1]};
          v = cfma(u, w, v);
        }
        return v;
      };
      const cpx<double> xab = X(ra, cb), xba = X(cb, ra);
      cpx<double> f = {0.5 * (xab.re - xba.re), 0.5 * (xab.im + xba.im)};
      if (ra == cb) {  // minus tr(X - X^dag) / 6 = i Im tr(X) / 3
        double imtr = 0.0;
#pragma unroll
        for (int k = 0; k < 3; k++) imtr += X(k, k).im;
        f.im -= imtr / 3.0;
      }
      const long site = (((long)t * L2 + z) * L1 + y) * L0 + x;
      cpx<double>* dst = a.F + (site * 4 + mu) * 9 + e;
      if (a.accumulate) f = cadd(*dst, f);
      *dst = f;
    }
  }
}

hipError_t launch_force(const void* chi_own, const void* psi_own, const void* chi_nb, const void* psi_nb,
                        const void* links, void* F, int par, int Ns, int bc_t, int accumulate, const Geom& g,
                        hipStream_t st) {
  ForceArgs a;
  a.chi_own = chi_own;
  a.psi_own = psi_own;
  a.chi_nb = chi_nb;
  a.psi_nb = psi_nb;
  a.links = links;
  a.F = reinterpret_cast<cpx<double>*>(F);
  for (int d = 0; d < 4; d++) a.L[d] = g.L[d];
  a.h = (int)g.h;
  a.Ns = Ns;
  a.par = par;
  a.bc_t = bc_t;
  a.accumulate = accumulate;
  if (Ns < 4 || Ns > 32 || (Ns & (Ns - 1))) return hipErrorInvalidValue;
  const int spb = 256 / Ns;
  const dim3 grid((unsigned)((g.h + spb - 1) / spb));
  hipLaunchKernelGGL(force_kernel, grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace odwf
