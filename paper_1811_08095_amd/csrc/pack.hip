// Layout kernels: canonical complex128 fields <-> internal even/odd halves.
//
// Canonical spinor: [rhs][s][t][z][y][x][spin 4][colour 3] complex128.
// Canonical gauge:  [t][z][y][x][mu][3][3] complex128, U_mu(x) links x to x + mu.
// Internal half of parity p: site j = ((t * Lz + z) * Ly + y) * (Lx / 2) + x / 2
// over the sites with (x + y + z + t) mod 2 = p; spinor chunks as described in
// dev_common.h; links per output parity [j][8][...] with directions 0-3 the
// forward links U_mu(x) and 4-7 the backward links U_mu(x - mu)^dag, FP64 as 9
// complex doubles, reduced precision as rows 0 and 1 (12 floats).
#include "dev_common.h"
#include "kernels.h"

namespace odwf {

__device__ __forceinline__ long full_index(long j, int par, const int* L, int& t_out) {
  const int hx = L[0] >> 1;
  const int xh = (int)(j % hx);
  long rest = j / hx;
  const int y = (int)(rest % L[1]);
  rest /= L[1];
  const int z = (int)(rest % L[2]);
  const int t = (int)(rest / L[2]);
  const int x = 2 * xh + ((y + z + t + par) & 1);
  t_out = t;
  return (((long)t * L[2] + z) * L[1] + y) * L[0] + x;
}

struct GeomK {
  int L[4];
  long V, h;
};

template <class P>
__global__ void pack_spinor_kernel(const double2* __restrict__ canon, int r0, void* out,
                                   float* out_sc, int par, int nrhs, int Ns, GeomK g) {
  using R = typename P::real;
  const long n = g.h * nrhs * Ns;
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
    const int s = (int)(k % Ns);
    const int r = (int)((k / Ns) % nrhs);
    const long j = k / ((long)Ns * nrhs);
    int t;
    const long i = full_index(j, par, g.L, t);
    const double2* src = canon + ((((long)(r0 + r) * Ns + s) * g.V + i) * 12);
    cpx<R> v[12];
#pragma unroll
    for (int c = 0; c < 12; c++) {
      double2 z = src[c];
      v[c] = {(R)z.x, (R)z.y};
    }
    store_site<P>(out, out_sc, j, r, s, nrhs, Ns, v);
  }
}

template <class P>
__global__ void unpack_spinor_kernel(const void* in, const float* in_sc, double2* __restrict__ canon,
                                     int r0, int par, int nrhs, int Ns, GeomK g) {
  using R = typename P::real;
  const long n = g.h * nrhs * Ns;
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
    const int s = (int)(k % Ns);
    const int r = (int)((k / Ns) % nrhs);
    const long j = k / ((long)Ns * nrhs);
    int t;
    const long i = full_index(j, par, g.L, t);
    double2* dst = canon + ((((long)(r0 + r) * Ns + s) * g.V + i) * 12);
    cpx<R> v[12];
    load_site<P>(in, in_sc, j, r, s, nrhs, Ns, v);
#pragma unroll
    for (int c = 0; c < 12; c++) dst[c] = make_double2((double)v[c].re, (double)v[c].im);
  }
}

__global__ void zero_canon_parity_kernel(double2* __restrict__ canon, int r0, int par, int nrhs,
                                         int Ns, GeomK g) {
  const long n = g.h * nrhs * Ns;
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
    const int s = (int)(k % Ns);
    const int r = (int)((k / Ns) % nrhs);
    const long j = k / ((long)Ns * nrhs);
    int t;
    const long i = full_index(j, par, g.L, t);
    double2* dst = canon + ((((long)(r0 + r) * Ns + s) * g.V + i) * 12);
#pragma unroll
    for (int c = 0; c < 12; c++) dst[c] = make_double2(0.0, 0.0);
  }
}

__global__ void pack_gauge_kernel(const double2* __restrict__ canon, void* out, int par, int prec,
                                  GeomK g) {
  const long n = g.h * 8;
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
    const int dir = (int)(k % 8);
    const long j = k / 8;
    int t;
    const long i = full_index(j, par, g.L, t);
    const int mu = dir & 3;
    double2 m[9];
    if (dir < 4) {
      const double2* u = canon + (i * 4 + mu) * 9;
#pragma unroll
      for (int q = 0; q < 9; q++) m[q] = u[q];
    } else {
      // neighbour x - mu (periodic; the boundary factor is applied by the kernel)
      long c[4];
      long rem = i;
      for (int d = 0; d < 4; d++) {
        c[d] = rem % g.L[d];
        rem /= g.L[d];
      }
      c[mu] = c[mu] == 0 ? g.L[mu] - 1 : c[mu] - 1;
      const long ib = ((c[3] * g.L[2] + c[2]) * g.L[1] + c[1]) * g.L[0] + c[0];
      const double2* u = canon + (ib * 4 + mu) * 9;
#pragma unroll
      for (int a = 0; a < 3; a++)
#pragma unroll
        for (int b = 0; b < 3; b++) {
          double2 v = u[b * 3 + a];
          m[a * 3 + b] = make_double2(v.x, -v.y);
        }
    }
    if (prec == PREC64) {
      double2* o = reinterpret_cast<double2*>(out) + k * 9;
#pragma unroll
      for (int q = 0; q < 9; q++) o[q] = m[q];
    } else {
      float2* o = reinterpret_cast<float2*>(out) + k * 6;
#pragma unroll
      for (int q = 0; q < 6; q++) o[q] = make_float2((float)m[q].x, (float)m[q].y);
    }
  }
}

// boundary maps of the effective 4D operator, on canonical fields:
// embed: 5D [r][s][site][spin][colour] from 4D [r][site][spin][colour], the
//   chirality-minus spins (2, 3) into slice 0, the chirality-plus spins (0, 1)
//   into slice Ns - 1, zeros elsewhere;
// project: 4D from 5D, chirality-plus spins of slice Ns - 1 and chirality-minus
//   spins of slice 0 (the pair of slices the m_q boundary term couples)
__global__ void boundary_embed_kernel(const double2* __restrict__ q, double2* __restrict__ f, int nrhs,
                                      int Ns, long V) {
  const long n = (long)nrhs * Ns * V * 12;
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
    const int c = (int)(k % 12);
    const long site = (k / 12) % V;
    const int s = (int)((k / (12 * V)) % Ns);
    const long r = k / (12 * V * Ns);
    const bool plus = c < 6;
    const bool take = (s == 0 && !plus) || (s == Ns - 1 && plus);
    f[k] = take ? q[(r * V + site) * 12 + c] : make_double2(0.0, 0.0);
  }
}

__global__ void boundary_project_kernel(const double2* __restrict__ f, double2* __restrict__ q, int nrhs,
                                        int Ns, long V) {
  const long n = (long)nrhs * V * 12;
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
    const int c = (int)(k % 12);
    const long site = (k / 12) % V;
    const long r = k / (12 * V);
    const int s = c < 6 ? Ns - 1 : 0;
    q[k] = f[((r * Ns + s) * V + site) * 12 + c];
  }
}

static GeomK gk(const Geom& g) {
  GeomK k;
  for (int d = 0; d < 4; d++) k.L[d] = g.L[d];
  k.V = g.V;
  k.h = g.h;
  return k;
}

static dim3 grid_for(long n, int block) {
  long b = (n + block - 1) / block;
  if (b > 65535L * 16) b = 65535L * 16;
  if (b < 1) b = 1;
  return dim3((unsigned)b);
}

hipError_t launch_pack_spinor(int prec, const void* canon, int r0, void* out, float* out_sc, int par,
                              int nrhs, int Ns, const Geom& g, hipStream_t st) {
  const long n = g.h * nrhs * Ns;
  const dim3 gr = grid_for(n, 256);
  const double2* c = reinterpret_cast<const double2*>(canon);
  switch (prec) {
    case PREC64: hipLaunchKernelGGL(pack_spinor_kernel<SP64>, gr, dim3(256), 0, st, c, r0, out, out_sc, par, nrhs, Ns, gk(g)); break;
    case PREC32: hipLaunchKernelGGL(pack_spinor_kernel<SP32>, gr, dim3(256), 0, st, c, r0, out, out_sc, par, nrhs, Ns, gk(g)); break;
    case PREC16: hipLaunchKernelGGL(pack_spinor_kernel<SP16>, gr, dim3(256), 0, st, c, r0, out, out_sc, par, nrhs, Ns, gk(g)); break;
    case PRECB16: hipLaunchKernelGGL(pack_spinor_kernel<SPB16>, gr, dim3(256), 0, st, c, r0, out, out_sc, par, nrhs, Ns, gk(g)); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_unpack_spinor(int prec, const void* in, const float* in_sc, void* canon, int r0,
                                int par, int nrhs, int Ns, const Geom& g, hipStream_t st) {
  const long n = g.h * nrhs * Ns;
  const dim3 gr = grid_for(n, 256);
  double2* c = reinterpret_cast<double2*>(canon);
  switch (prec) {
    case PREC64: hipLaunchKernelGGL(unpack_spinor_kernel<SP64>, gr, dim3(256), 0, st, in, in_sc, c, r0, par, nrhs, Ns, gk(g)); break;
    case PREC32: hipLaunchKernelGGL(unpack_spinor_kernel<SP32>, gr, dim3(256), 0, st, in, in_sc, c, r0, par, nrhs, Ns, gk(g)); break;
    case PREC16: hipLaunchKernelGGL(unpack_spinor_kernel<SP16>, gr, dim3(256), 0, st, in, in_sc, c, r0, par, nrhs, Ns, gk(g)); break;
    case PRECB16: hipLaunchKernelGGL(unpack_spinor_kernel<SPB16>, gr, dim3(256), 0, st, in, in_sc, c, r0, par, nrhs, Ns, gk(g)); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_zero_canon_parity(void* canon, int r0, int par, int nrhs, int Ns, const Geom& g,
                                    hipStream_t st) {
  const long n = g.h * nrhs * Ns;
  hipLaunchKernelGGL(zero_canon_parity_kernel, grid_for(n, 256), dim3(256), 0, st,
                     reinterpret_cast<double2*>(canon), r0, par, nrhs, Ns, gk(g));
  return hipGetLastError();
}

hipError_t launch_boundary_embed(const void* q, void* f, int nrhs, int Ns, const Geom& g, hipStream_t st) {
  const long n = (long)nrhs * Ns * g.V * 12;
  hipLaunchKernelGGL(boundary_embed_kernel, grid_for(n, 256), dim3(256), 0, st,
                     reinterpret_cast<const double2*>(q), reinterpret_cast<double2*>(f), nrhs, Ns, g.V);
  return hipGetLastError();
}

hipError_t launch_boundary_project(const void* f, void* q, int nrhs, int Ns, const Geom& g, hipStream_t st) {
  const long n = (long)nrhs * g.V * 12;
  hipLaunchKernelGGL(boundary_project_kernel, grid_for(n, 256), dim3(256), 0, st,
                     reinterpret_cast<const double2*>(f), reinterpret_cast<double2*>(q), nrhs, Ns, g.V);
  return hipGetLastError();
}

hipError_t launch_pack_gauge(const void* canon, void* out, int par, int prec, const Geom& g,
                             hipStream_t st) {
  const long n = g.h * 8;
  hipLaunchKernelGGL(pack_gauge_kernel, grid_for(n, 256), dim3(256), 0, st,
                     reinterpret_cast<const double2*>(canon), out, par, prec, gk(g));
  return hipGetLastError();
}

}  // namespace odwf
