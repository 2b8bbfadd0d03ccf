// Even-odd hopping kernel ("Dslash") of the optimal domain-wall operator with
// fused fifth-dimension epilogues and fused CG updates.
//
// Computes, for every site x of the output parity, right-hand side r and slice s,
//     (W psi)(x, s) = -1/2 sum_mu [ (1 - gamma_mu) U_mu(x) psi(x + mu, s)
//                                 + (1 + gamma_mu) U_mu(x - mu)^dag psi(x - mu, s) ]
// (the hopping part of the 4D Wilson operator D_w of §2 with H = H_w; the
// adjoint W^dag swaps the two projectors), hops across the t boundary
// multiplied by bc_t, then
//     y = c_h * P_h(W psi) + c_x * P_x(x_site),   out = P_o(y)
// where P_h, P_x, P_o are fifth-dimension programs (A^{-1}, A^{-dag}, A^dag, ...
// as products of cyclic bidiagonal factors), and optionally a fused CG step.
//
// Thread layout: a block holds spb sites of the output parity; each site has
// nrhs * Ns lanes (s fastest) that read consecutive 16-byte chunks of every
// neighbour.  The 8 links of the block's sites are staged once in LDS and
// shared by all nrhs * Ns lanes of a site (links are stored per output parity
// as [site][8][...] with directions 0-3 forward U_mu(x) and 4-7 backward
// U_mu(x - mu)^dag).  Fifth-dimension programs run in LDS on columns
// (site, r, colour-spin component) of Ns values.  No MFMA: the stencil is a
// string of 3x3 complex mat-vecs and is bound by HBM bandwidth.
#include "dev_common.h"
#include "kernels.h"

namespace odwf {

// --- link formats ---------------------------------------------------------

template <class P>
struct LinkFmt;
// FP64: 18 reals = 9 complex doubles per matrix
template <>
struct LinkFmt<SP64> {
  static constexpr int REALS = 18;
  using R = double;
};
// reduced precisions: 12 reals (rows 0, 1) as floats, row 2 rebuilt as
// conj(row0 x row1), valid for SU(3)
struct LinkF12 {
  static constexpr int REALS = 12;
  using R = float;
};
template <>
struct LinkFmt<SP32> : LinkF12 {};
template <>
struct LinkFmt<SP16> : LinkF12 {};
template <>
struct LinkFmt<SPB16> : LinkF12 {};

// stage the links of `nsb` sites starting at j0 into LDS as 9 complex per matrix
template <class P>
__device__ __forceinline__ void stage_links(const void* links, long j0, int nsb,
                                            cpx<typename P::real>* lnk) {
  using R = typename P::real;
  const int nmat = nsb * 8;
  if constexpr (LinkFmt<P>::REALS == 18) {
    // flat copy of 16-byte chunks (one complex double each)
    const uint4* src = reinterpret_cast<const uint4*>(links) + j0 * 8 * 9;
    for (int q = threadIdx.x; q < nmat * 9; q += blockDim.x) {
      uint4 v = src[q];
      cpx<double> z;
      unpack_chunk<SP64>(v, &z);
      lnk[q] = z;
    }
  } else {
    const float4* src = reinterpret_cast<const float4*>(links) + j0 * 8 * 3;
    for (int m = threadIdx.x; m < nmat; m += blockDim.x) {
      float4 a = src[m * 3 + 0], b = src[m * 3 + 1], c = src[m * 3 + 2];
      cpx<float> u[6] = {{a.x, a.y}, {a.z, a.w}, {b.x, b.y}, {b.z, b.w}, {c.x, c.y}, {c.z, c.w}};
      cpx<R>* d = lnk + m * 9;
#pragma unroll
      for (int k = 0; k < 6; k++) d[k] = u[k];
      // row2[a] = conj(row0[b] row1[c] - row0[c] row1[b]), (a, b, c) cyclic
#pragma unroll
      for (int a0 = 0; a0 < 3; a0++) {
        const int b0 = (a0 + 1) % 3, c0 = (a0 + 2) % 3;
        cpx<float> t = csub(cmul(u[b0], u[3 + c0]), cmul(u[c0], u[3 + b0]));
        d[6 + a0] = {t.re, -t.im};
      }
    }
  }
}

// multiplication by f in {+1, -1, +i, -i} (codes 0..3)
template <int CODE, class R>
__device__ __forceinline__ cpx<R> mulf(cpx<R> z) {
  if constexpr (CODE == 0) return z;
  if constexpr (CODE == 1) return {-z.re, -z.im};
  if constexpr (CODE == 2) return {-z.im, z.re};
  return {z.im, -z.re};
}
template <int CODE>
struct ConjCode {
  static constexpr int v = CODE == 2 ? 3 : (CODE == 3 ? 2 : CODE);
};

// chiral basis: gamma_mu = [[0, B_mu], [B_mu^dag, 0]], row a of B_mu has one
// entry f_a at column p_a:
//   mu = x: p = (1, 0), f = (-i, -i);   mu = y: p = (1, 0), f = (-1, +1)
//   mu = z: p = (0, 1), f = (-i, +i);   mu = t: p = (0, 1), f = (+1, +1)
template <int MU>
struct GammaB;
template <>
struct GammaB<0> {
  static constexpr int p0 = 1, p1 = 0, f0 = 3, f1 = 3;
};
template <>
struct GammaB<1> {
  static constexpr int p0 = 1, p1 = 0, f0 = 1, f1 = 0;
};
template <>
struct GammaB<2> {
  static constexpr int p0 = 0, p1 = 1, f0 = 3, f1 = 2;
};
template <>
struct GammaB<3> {
  static constexpr int p0 = 0, p1 = 1, f0 = 0, f1 = 0;
};

// (1 - SIG gamma_mu) psi = [h; -SIG B^dag h], h = psi_up - SIG B psi_dn.
// Computes the half spinor h (2 spins x 3 colours).
template <int MU, int SIG, class R>
__device__ __forceinline__ void project(const cpx<R> (&psi)[12], cpx<R> (&h)[6]) {
  using B = GammaB<MU>;
#pragma unroll
  for (int c = 0; c < 3; c++) {
    cpx<R> t0 = mulf<B::f0>(psi[(2 + B::p0) * 3 + c]);
    cpx<R> t1 = mulf<B::f1>(psi[(2 + B::p1) * 3 + c]);
    if constexpr (SIG > 0) {
      h[c] = csub(psi[c], t0);
      h[3 + c] = csub(psi[3 + c], t1);
    } else {
      h[c] = cadd(psi[c], t0);
      h[3 + c] = cadd(psi[3 + c], t1);
    }
  }
}

// acc += [g; -SIG B^dag g]; (B^dag g)_b = conj(f_{p_b}) g_{p_b}
template <int MU, int SIG, class R>
__device__ __forceinline__ void reconstruct(const cpx<R> (&g)[6], cpx<R> (&acc)[12]) {
  using B = GammaB<MU>;
  // p is an involution here: p_b = p0 for b = 0, p1 for b = 1
  constexpr int q0 = B::p0, q1 = B::p1;
  constexpr int fq0 = (q0 == 0) ? B::f0 : B::f1;
  constexpr int fq1 = (q1 == 0) ? B::f0 : B::f1;
#pragma unroll
  for (int c = 0; c < 3; c++) {
    acc[c] = cadd(acc[c], g[c]);
    acc[3 + c] = cadd(acc[3 + c], g[3 + c]);
    cpx<R> l0 = mulf<ConjCode<fq0>::v>(g[q0 * 3 + c]);
    cpx<R> l1 = mulf<ConjCode<fq1>::v>(g[q1 * 3 + c]);
    if constexpr (SIG > 0) {
      acc[6 + c] = csub(acc[6 + c], l0);
      acc[9 + c] = csub(acc[9 + c], l1);
    } else {
      acc[6 + c] = cadd(acc[6 + c], l0);
      acc[9 + c] = cadd(acc[9 + c], l1);
    }
  }
}

// g = U h for both spins of the half spinor
template <class R>
__device__ __forceinline__ void su3_mul(const cpx<R>* __restrict__ U, const cpx<R> (&h)[6],
                                        cpx<R> (&g)[6]) {
#pragma unroll
  for (int a = 0; a < 3; a++) {
    const cpx<R> u0 = U[a * 3 + 0], u1 = U[a * 3 + 1], u2 = U[a * 3 + 2];
#pragma unroll
    for (int sp = 0; sp < 2; sp++) {
      cpx<R> v = cmul(u0, h[sp * 3 + 0]);
      v = cfma(u1, h[sp * 3 + 1], v);
      v = cfma(u2, h[sp * 3 + 2], v);
      g[sp * 3 + a] = v;
    }
  }
}

// one hop: acc += [g; -SIG B^dag g] with g = U (psi_up - SIG B psi_dn)
template <int MU, int SIG, class R>
__device__ __forceinline__ void hop_one(const cpx<R> (&psi)[12], const cpx<R>* U, cpx<R> (&acc)[12]) {
  cpx<R> h[6], g[6];
  project<MU, SIG>(psi, h);
  su3_mul(U, h, g);
  reconstruct<MU, SIG>(g, acc);
}

// first site of this block under the configured traversal
__device__ __forceinline__ long block_first_site(const HopArgs& a) {
  int lb = blockIdx.x;
  if (a.xcd) {
    // hardware dispatches block b to XCD b % 8; give XCD x the contiguous
    // logical range [start(x), start(x) + count(x))
    const int q = a.nblocks >> 3, rem = a.nblocks & 7;
    const int x = lb & 7, k = lb >> 3;
    lb = x * q + min(x, rem) + k;
  }
  if (a.tile_y > 0) {
    const int hx = a.L[0] >> 1;
    const int nseg = hx / a.spb;
    int rest = lb;
    const int seg = rest % nseg;
    rest /= nseg;
    const int yi = rest % a.tile_y;
    rest /= a.tile_y;
    const int zi = rest % a.tile_z;
    rest /= a.tile_z;
    const int t = rest % a.L[3];
    rest /= a.L[3];
    const int nty = a.L[1] / a.tile_y;
    const int y = (rest % nty) * a.tile_y + yi;
    const int z = (rest / nty) * a.tile_z + zi;
    return (((long)t * a.L[2] + z) * a.L[1] + y) * hx + (long)seg * a.spb;
  }
  return (long)lb * a.spb;
}

#ifndef ODWF_HOP_GROUP64
#define ODWF_HOP_GROUP64 1
#endif
#ifndef ODWF_HOP_GROUP32
#define ODWF_HOP_GROUP32 2
#endif

// neighbour loads issued together before any of them is used: enough bytes
// in flight per wave to cover HBM latency at the occupancy the kernel reaches
template <class P>
struct HopGroup {
  static constexpr int G = sizeof(typename P::real) == 8 ? ODWF_HOP_GROUP64 : ODWF_HOP_GROUP32;
};

// minimum waves per SIMD the register allocation must allow
template <class P, bool PLAIN>
struct HopWaves {
  static constexpr int W = sizeof(typename P::real) == 8 ? (PLAIN ? 2 : 1) : (PLAIN ? 4 : 2);
};

template <class P, int NS, bool DAG, bool PLAIN>
__global__ void __launch_bounds__(256, (HopWaves<P, PLAIN>::W)) hop_kernel(const HopArgs a) {
  using R = typename P::real;
  extern __shared__ __align__(16) unsigned char smem[];
  const int nrhs = a.nrhs;
  const int inner = nrhs * NS;
  const int tid = threadIdx.x;
  const int sl = tid / inner;
  const int lr = tid - sl * inner;
  const int r = lr / NS;
  const int s = lr - r * NS;
  if (!gate_any(a.gate, a.gate_mode, nrhs)) return;  // whole block idle
  const long j0 = block_first_site(a);
  const int nsb = (int)min((long)a.spb, (long)a.h - j0);
  // padded threads have sl >= spb >= nsb; gated-off right-hand sides do no work
  const bool valid = sl < nsb && gate_on(a.gate, a.gate_mode, r);
  const long j = j0 + sl;
  constexpr int NSP = NS + 1;

  // LDS carve-up: links, then (aliased) the column buffer; reduction scratch
  // links and the column buffer live in separate regions, so an x term can be
  // transformed in LDS while the links are staged and used
  const size_t lnk_n = (size_t)a.spb * 8 * 9;
  const size_t buf_n = PLAIN ? 0 : (size_t)a.spb * nrhs * 12 * NSP;
  cpx<R>* lnk = reinterpret_cast<cpx<R>*>(smem);
  cpx<R>* buf = lnk + lnk_n;
  const size_t region = (lnk_n + buf_n) * sizeof(cpx<R>);
  R* kap = reinterpret_cast<R*>(smem + region);
  double* red = reinterpret_cast<double*>(smem + ((region + MAXRHS * sizeof(R) + 15) & ~size_t(15)));
  double* rtmp = red + blockDim.x;
  const R* coef = reinterpret_cast<const R*>(a.coef);
  if (!PLAIN && tid < nrhs) kap[tid] = (R)a.kappa[tid];
  stage_links<P>(a.links, j0, nsb, lnk);

  cpx<R> xv[12];
  const bool has_x = !PLAIN && a.xin != nullptr;
  // x term with its own fifth-dimension program: transform it in LDS before the
  // hop, so no column pass runs while the hop accumulators are live
  const bool x_first = has_x && a.prog_x.n > 0;
  if (x_first) {
    if (valid) {
      load_site<P>(a.xin, a.xin_sc, j, r, s, nrhs, NS, xv);
      cpx<R>* b = buf + ((size_t)(sl * nrhs + r) * 12) * NSP + s;
#pragma unroll
      for (int c = 0; c < 12; c++) b[c * NSP] = xv[c];
    }
    __syncthreads();
    column_pass_lds<R, NS>(buf, nsb, nrhs, a.prog_x, coef, kap);
  }
  __syncthreads();

  cpx<R> acc[12];
#pragma unroll
  for (int c = 0; c < 12; c++) acc[c] = {R(0), R(0)};

  if (valid) {
    const int L0 = a.L[0], L1 = a.L[1], L2 = a.L[2], L3 = a.L[3];
    const int hx = L0 >> 1;
    // site coordinates: when a block lies inside one x-row (always for the
    // tiled traversal) y, z, t are block-uniform and only x varies by lane
    int x, y, z, t;
    if (hx % a.spb == 0) {
      const int xh0 = (int)(j0 % hx);
      long rest = j0 / hx;
      y = (int)(rest % L1);
      rest /= L1;
      z = (int)(rest % L2);
      t = (int)(rest / L2);
      x = 2 * (xh0 + sl) + ((y + z + t + a.out_par) & 1);
    } else {
      const int xh = (int)(j % hx);
      long rest = j / hx;
      y = (int)(rest % L1);
      rest /= L1;
      z = (int)(rest % L2);
      t = (int)(rest / L2);
      x = 2 * xh + ((y + z + t + a.out_par) & 1);
    }
    const cpx<R>* U = lnk + (size_t)sl * 8 * 9;
    const bool flip_f = a.bc_t < 0 && t + 1 == L3;  // forward t hop wraps
    const bool flip_b = a.bc_t < 0 && t == 0;       // backward t hop wraps
    constexpr int G = HopGroup<P>::G;
    // direction order: +x, -x, +y, -y, ... (4-7 are the backward hops)
#pragma unroll 1
    for (int g0 = 0; g0 < 8; g0 += G) {
      cpx<R> psi[G][12];
#pragma unroll
      for (int k = 0; k < G; k++) {
        const int dir = ((g0 + k) >> 1) | (((g0 + k) & 1) << 2);  // 0,4,1,5,2,6,3,7
        const int mu = dir & 3;
        const bool fwd = dir < 4;
        int xx = x, yy = y, zz = z, tt = t;
        if (mu == 0) xx = fwd ? (x + 1 == L0 ? 0 : x + 1) : (x == 0 ? L0 - 1 : x - 1);
        if (mu == 1) yy = fwd ? (y + 1 == L1 ? 0 : y + 1) : (y == 0 ? L1 - 1 : y - 1);
        if (mu == 2) zz = fwd ? (z + 1 == L2 ? 0 : z + 1) : (z == 0 ? L2 - 1 : z - 1);
        if (mu == 3) tt = fwd ? (t + 1 == L3 ? 0 : t + 1) : (t == 0 ? L3 - 1 : t - 1);
        const long nj = (((long)tt * L2 + zz) * L1 + yy) * hx + (xx >> 1);
        load_site_cached<P>(a.in, a.in_sc, nj, r, s, nrhs, NS, psi[k]);
      }
#pragma unroll
      for (int k = 0; k < G; k++) {
        const int dir = ((g0 + k) >> 1) | (((g0 + k) & 1) << 2);
        const bool fwd = dir < 4;
        if ((dir == 3 && flip_f) || (dir == 7 && flip_b)) {
#pragma unroll
          for (int c = 0; c < 12; c++) psi[k][c] = {-psi[k][c].re, -psi[k][c].im};
        }
        // forward hop: (1 - gamma) for W, (1 + gamma) for W^dag; backward swapped
        const bool minus = fwd != DAG;
        switch (dir & 3) {
          case 0: if (minus) hop_one<0, +1>(psi[k], U + dir * 9, acc); else hop_one<0, -1>(psi[k], U + dir * 9, acc); break;
          case 1: if (minus) hop_one<1, +1>(psi[k], U + dir * 9, acc); else hop_one<1, -1>(psi[k], U + dir * 9, acc); break;
          case 2: if (minus) hop_one<2, +1>(psi[k], U + dir * 9, acc); else hop_one<2, -1>(psi[k], U + dir * 9, acc); break;
          default: if (minus) hop_one<3, +1>(psi[k], U + dir * 9, acc); else hop_one<3, -1>(psi[k], U + dir * 9, acc); break;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 12; c++) acc[c] = cscale(R(-0.5), acc[c]);
  }
  if constexpr (PLAIN) {
    if (valid) store_site<P>(a.out, a.out_sc, j, r, s, nrhs, NS, acc);
    return;
  }

  // ---- fifth-dimension column passes --------------------------------------
  auto column_pass = [&](const M5Prog& prog, cpx<R>(&v)[12]) {
    __syncthreads();
    if (valid) {
      cpx<R>* b = buf + ((size_t)(sl * nrhs + r) * 12) * NSP + s;
#pragma unroll
      for (int c = 0; c < 12; c++) b[c * NSP] = v[c];
    }
    __syncthreads();
    column_pass_lds<R, NS>(buf, nsb, nrhs, prog, coef, kap);
    __syncthreads();
    if (valid) {
      const cpx<R>* b = buf + ((size_t)(sl * nrhs + r) * 12) * NSP + s;
#pragma unroll
      for (int c = 0; c < 12; c++) v[c] = b[c * NSP];
    }
  };

  if (a.prog_h.n > 0) column_pass(a.prog_h, acc);  // never together with x_first
  if (has_x && valid) {
    if (x_first) {
      const cpx<R>* b = buf + ((size_t)(sl * nrhs + r) * 12) * NSP + s;
#pragma unroll
      for (int c = 0; c < 12; c++) xv[c] = b[c * NSP];
    } else {
      load_site<P>(a.xin, a.xin_sc, j, r, s, nrhs, NS, xv);
    }
  }
  if (has_x) {
    const R ch = (R)a.c_h, cx = (R)a.c_x;
#pragma unroll
    for (int c = 0; c < 12; c++) acc[c] = cadd(cscale(ch, acc[c]), cscale(cx, xv[c]));
  } else if (a.c_h != 1.0) {
    const R ch = (R)a.c_h;
#pragma unroll
    for (int c = 0; c < 12; c++) acc[c] = cscale(ch, acc[c]);
  }

  const int cgmode = a.partial ? (a.cg_r ? 2 : (a.cg_p ? 3 : 1)) : 0;
  double nval = 0.0;
  if (cgmode == 1 && valid) {
#pragma unroll
    for (int c = 0; c < 12; c++) nval += (double)cnorm2(acc[c]);
  }
  if (a.prog_o.n > 0) column_pass(a.prog_o, acc);

  if (cgmode == 3 && valid) {  // residual: out = f - y
    cpx<R> f[12];
    load_site<P>(a.cg_p, a.cg_p_sc, j, r, s, nrhs, NS, f);
#pragma unroll
    for (int c = 0; c < 12; c++) {
      acc[c] = csub(f[c], acc[c]);
      nval += (double)cnorm2(acc[c]);
    }
  }
  if (cgmode == 2) {
    if (valid && a.scal[r].active) {
      const R al = (R)a.scal[r].alpha;
      {  // r -= alpha N p, |r|^2
        cpx<R> rv[12];
        load_site<P>(a.cg_r, a.cg_r_sc, j, r, s, nrhs, NS, rv);
#pragma unroll
        for (int c = 0; c < 12; c++) {
          rv[c] = csub(rv[c], cscale(al, acc[c]));
          nval += (double)cnorm2(rv[c]);
        }
        store_site<P>(a.cg_r, a.cg_r_sc, j, r, s, nrhs, NS, rv);
      }
      {  // x += alpha p
        cpx<R> xx[12], pv[12];
        load_site<P>(a.cg_x, a.cg_x_sc, j, r, s, nrhs, NS, xx);
        load_site<P>(a.cg_p, a.cg_p_sc, j, r, s, nrhs, NS, pv);
#pragma unroll
        for (int c = 0; c < 12; c++) xx[c] = cadd(xx[c], cscale(al, pv[c]));
        store_site<P>(a.cg_x, a.cg_x_sc, j, r, s, nrhs, NS, xx);
      }
    }
  } else if (valid && a.out) {
    store_site<P>(a.out, a.out_sc, j, r, s, nrhs, NS, acc);
  }

  if (cgmode) {
    red[tid] = valid ? nval : 0.0;
    block_reduce_rhs(
        red, blockDim.x, nrhs, [&](int k) { return (k % inner) / NS; }, rtmp, a.partial);
  }
}

template <class P, int NS>
static size_t hop_smem(int spb, int nrhs, int block, bool plain) {
  using R = typename P::real;
  const size_t lnk_n = (size_t)spb * 8 * 9;
  const size_t buf_n = plain ? 0 : (size_t)spb * nrhs * 12 * (NS + 1);
  const size_t region = (lnk_n + buf_n) * sizeof(cpx<R>);
  size_t off = (region + MAXRHS * sizeof(R) + 15) & ~size_t(15);
  return off + (size_t)(block + 16 * MAXRHS) * sizeof(double);
}

template <class P, int NS>
static hipError_t launch_hop_t(HopArgs a, int dag, hipStream_t st) {
  const int inner = a.nrhs * NS;
  if (inner > 256 || a.nrhs > MAXRHS) return hipErrorInvalidValue;
  a.spb = 256 / inner;
  const int block = (a.spb * inner + 63) & ~63;  // whole waves, <= 256
  a.nblocks = (int)((a.h + a.spb - 1) / a.spb);
  const bool plain = a.prog_h.n == 0 && a.prog_o.n == 0 && a.xin == nullptr && a.partial == nullptr &&
                     a.c_h == 1.0;
  const size_t sm = hop_smem<P, NS>(a.spb, a.nrhs, block, plain);
  if (plain) {
    if (dag) hipLaunchKernelGGL((hop_kernel<P, NS, true, true>), dim3(a.nblocks), dim3(block), sm, st, a);
    else hipLaunchKernelGGL((hop_kernel<P, NS, false, true>), dim3(a.nblocks), dim3(block), sm, st, a);
  } else {
    if (dag) hipLaunchKernelGGL((hop_kernel<P, NS, true, false>), dim3(a.nblocks), dim3(block), sm, st, a);
    else hipLaunchKernelGGL((hop_kernel<P, NS, false, false>), dim3(a.nblocks), dim3(block), sm, st, a);
  }
  return hipGetLastError();
}

int hop_nblocks(int h, int nrhs, int Ns) {
  const int inner = nrhs * Ns;
  const int spb = inner >= 256 ? 1 : 256 / inner;
  return (h + spb - 1) / spb;
}

template <class P>
static hipError_t launch_hop_p(const HopArgs& a, int Ns, int dag, hipStream_t st) {
  switch (Ns) {
    case 4: return launch_hop_t<P, 4>(a, dag, st);
    case 8: return launch_hop_t<P, 8>(a, dag, st);
    case 16: return launch_hop_t<P, 16>(a, dag, st);
    case 32: return launch_hop_t<P, 32>(a, dag, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_hop(const HopArgs& a, int prec, int Ns, hipStream_t st) {
  switch (prec) {
    case PREC64: return launch_hop_p<SP64>(a, Ns, a.dag, st);
    case PREC32: return launch_hop_p<SP32>(a, Ns, a.dag, st);
    case PREC16: return launch_hop_p<SP16>(a, Ns, a.dag, st);
    case PRECB16: return launch_hop_p<SPB16>(a, Ns, a.dag, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace odwf
