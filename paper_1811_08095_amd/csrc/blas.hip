// BLAS-1 kernels on even/odd half fields and the CG scalar finalisation.
//
// Threads map to 5D sites (j, r, s) with s fastest and a block size that is a
// multiple of nrhs * Ns, so every thread keeps one right-hand side across its
// grid-stride loop and per-right-hand-side reductions stay deterministic:
// per-block partial sums (fixed order) followed by a one-block finalisation
// that sums the partials in a fixed tree.  All accumulations are FP64.
#include "dev_common.h"
#include "kernels.h"

namespace odwf {

static inline int vec_spb(int nrhs, int Ns) {
  const int inner = nrhs * Ns;
  return inner >= 256 ? 1 : 256 / inner;
}

int vec_nblocks(long h, int nrhs, int Ns) {
  const int spb = vec_spb(nrhs, Ns);
  long nb = (h + spb - 1) / spb;
  if (nb > 2048) nb = 2048;
  return (int)nb;
}

template <class P>
__global__ void vec_zero_kernel(void* v, float* sc, const CGScal* gate, int gate_mode, long h, int nrhs,
                                int Ns) {
  using R = typename P::real;
  const int inner = nrhs * Ns;
  const int spb = blockDim.x / inner;
  const int sl = threadIdx.x / inner, lr = threadIdx.x % inner, r = lr / Ns, s = lr % Ns;
  if (!gate_on(gate, gate_mode, r)) return;
  cpx<R> z[12];
#pragma unroll
  for (int c = 0; c < 12; c++) z[c] = {R(0), R(0)};
  for (long j = (long)blockIdx.x * spb + sl; j < h; j += (long)gridDim.x * spb)
    store_site<P>(v, sc, j, r, s, nrhs, Ns, z);
}

template <class PS, class PD>
__global__ void vec_convert_kernel(const void* src, const float* src_sc, void* dst, float* dst_sc,
                                   int accumulate, const CGScal* gate, int gate_mode, long h, int nrhs,
                                   int Ns) {
  using RS = typename PS::real;
  using RD = typename PD::real;
  const int inner = nrhs * Ns;
  const int spb = blockDim.x / inner;
  const int sl = threadIdx.x / inner, lr = threadIdx.x % inner, r = lr / Ns, s = lr % Ns;
  if (!gate_on(gate, gate_mode, r)) return;
  for (long j = (long)blockIdx.x * spb + sl; j < h; j += (long)gridDim.x * spb) {
    cpx<RS> a[12];
    load_site<PS>(src, src_sc, j, r, s, nrhs, Ns, a);
    cpx<RD> b[12];
    if (accumulate) {
      load_site<PD>(dst, dst_sc, j, r, s, nrhs, Ns, b);
#pragma unroll
      for (int c = 0; c < 12; c++) b[c] = {b[c].re + (RD)a[c].re, b[c].im + (RD)a[c].im};
    } else {
#pragma unroll
      for (int c = 0; c < 12; c++) b[c] = {(RD)a[c].re, (RD)a[c].im};
    }
    store_site<PD>(dst, dst_sc, j, r, s, nrhs, Ns, b);
  }
}

// CG vector step after the scalars of the iteration are known:
//   x += alpha p   (for every right-hand side that iterated: alpha != 0, which
//                   includes one that converged at this iteration's beta)
//   p  = r + beta p (for the right-hand sides still active)
template <class P>
__global__ void vec_cg_step_kernel(const void* r_, const float* r_sc, void* p_, float* p_sc, void* x_,
                                   float* x_sc, const CGScal* scal, long h, int nrhs, int Ns) {
  using R = typename P::real;
  const int inner = nrhs * Ns;
  const int spb = blockDim.x / inner;
  const int sl = threadIdx.x / inner, lr = threadIdx.x % inner, r = lr / Ns, s = lr % Ns;
  const bool act = scal[r].active != 0;
  const double alpha = scal[r].alpha;
  if (!act && alpha == 0.0) return;
  const R al = (R)alpha, beta = (R)scal[r].beta;
  for (long j = (long)blockIdx.x * spb + sl; j < h; j += (long)gridDim.x * spb) {
    cpx<R> pv[12];
    load_site<P>(p_, p_sc, j, r, s, nrhs, Ns, pv);
    if (alpha != 0.0) {
      cpx<R> xv[12];
      load_site<P>(x_, x_sc, j, r, s, nrhs, Ns, xv);
#pragma unroll
      for (int c = 0; c < 12; c++) xv[c] = cadd(xv[c], cscale(al, pv[c]));
      store_site<P>(x_, x_sc, j, r, s, nrhs, Ns, xv);
    }
    if (act) {
      cpx<R> rv[12];
      load_site<P>(r_, r_sc, j, r, s, nrhs, Ns, rv);
#pragma unroll
      for (int c = 0; c < 12; c++) pv[c] = cadd(rv[c], cscale(beta, pv[c]));
      store_site<P>(p_, p_sc, j, r, s, nrhs, Ns, pv);
    }
  }
}

template <class P>
__global__ void vec_norm2_kernel(const void* v, const float* sc, double* partial, long h, int nrhs,
                                 int Ns) {
  using R = typename P::real;
  __shared__ double red[1024];
  const int inner = nrhs * Ns;
  const int spb = blockDim.x / inner;
  const int sl = threadIdx.x / inner, lr = threadIdx.x % inner, r = lr / Ns, s = lr % Ns;
  double acc = 0.0;
  if (sl < spb)
    for (long j = (long)blockIdx.x * spb + sl; j < h; j += (long)gridDim.x * spb) {
      cpx<R> a[12];
      load_site<P>(v, sc, j, r, s, nrhs, Ns, a);
#pragma unroll
      for (int c = 0; c < 12; c++) acc += (double)cnorm2(a[c]);
    }
  block_reduce_rhs(sl < spb ? acc : 0.0, Ns, spb, nrhs, red, partial, blockIdx.x);
}

#define ODWF_PREC_SWITCH(prec, KERNEL, ...)                                             \
  switch (prec) {                                                                       \
    case PREC64: hipLaunchKernelGGL(KERNEL<SP64>, __VA_ARGS__); break;                  \
    case PREC32: hipLaunchKernelGGL(KERNEL<SP32>, __VA_ARGS__); break;                  \
    case PREC16: hipLaunchKernelGGL(KERNEL<SP16>, __VA_ARGS__); break;                  \
    case PRECB16: hipLaunchKernelGGL(KERNEL<SPB16>, __VA_ARGS__); break;                \
    default: return hipErrorInvalidValue;                                               \
  }

hipError_t launch_vec_zero(int prec, void* v, float* sc, long h, int nrhs, int Ns, hipStream_t st,
                           const CGScal* gate, int gate_mode) {
  const int block = vec_spb(nrhs, Ns) * nrhs * Ns;
  const dim3 gr(vec_nblocks(h, nrhs, Ns));
  ODWF_PREC_SWITCH(prec, vec_zero_kernel, gr, dim3(block), 0, st, v, sc, gate, gate_mode, h, nrhs, Ns);
  return hipGetLastError();
}

template <class PS>
static hipError_t convert_to(int prec_dst, const void* src, const float* src_sc, void* dst,
                             float* dst_sc, int acc, const CGScal* gate, int gm, long h, int nrhs,
                             int Ns, hipStream_t st) {
  const int block = vec_spb(nrhs, Ns) * nrhs * Ns;
  const dim3 gr(vec_nblocks(h, nrhs, Ns));
  switch (prec_dst) {
    case PREC64: hipLaunchKernelGGL((vec_convert_kernel<PS, SP64>), gr, dim3(block), 0, st, src, src_sc, dst, dst_sc, acc, gate, gm, h, nrhs, Ns); break;
    case PREC32: hipLaunchKernelGGL((vec_convert_kernel<PS, SP32>), gr, dim3(block), 0, st, src, src_sc, dst, dst_sc, acc, gate, gm, h, nrhs, Ns); break;
    case PREC16: hipLaunchKernelGGL((vec_convert_kernel<PS, SP16>), gr, dim3(block), 0, st, src, src_sc, dst, dst_sc, acc, gate, gm, h, nrhs, Ns); break;
    case PRECB16: hipLaunchKernelGGL((vec_convert_kernel<PS, SPB16>), gr, dim3(block), 0, st, src, src_sc, dst, dst_sc, acc, gate, gm, h, nrhs, Ns); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_vec_convert(int prec_src, const void* src, const float* src_sc, int prec_dst,
                              void* dst, float* dst_sc, int accumulate, long h, int nrhs, int Ns,
                              hipStream_t st, const CGScal* gate, int gate_mode) {
  switch (prec_src) {
    case PREC64: return convert_to<SP64>(prec_dst, src, src_sc, dst, dst_sc, accumulate, gate, gate_mode, h, nrhs, Ns, st);
    case PREC32: return convert_to<SP32>(prec_dst, src, src_sc, dst, dst_sc, accumulate, gate, gate_mode, h, nrhs, Ns, st);
    case PREC16: return convert_to<SP16>(prec_dst, src, src_sc, dst, dst_sc, accumulate, gate, gate_mode, h, nrhs, Ns, st);
    case PRECB16: return convert_to<SPB16>(prec_dst, src, src_sc, dst, dst_sc, accumulate, gate, gate_mode, h, nrhs, Ns, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_vec_cg_step(int prec, const void* r, const float* r_sc, void* p, float* p_sc, void* x,
                              float* x_sc, const CGScal* scal, long h, int nrhs, int Ns, hipStream_t st) {
  const int block = vec_spb(nrhs, Ns) * nrhs * Ns;
  const dim3 gr(vec_nblocks(h, nrhs, Ns));
  ODWF_PREC_SWITCH(prec, vec_cg_step_kernel, gr, dim3(block), 0, st, r, r_sc, p, p_sc, x, x_sc, scal, h, nrhs,
                   Ns);
  return hipGetLastError();
}

hipError_t launch_vec_norm2(int prec, const void* v, const float* sc, double* partial, long h,
                            int nrhs, int Ns, int* nblocks_out, hipStream_t st) {
  const int block = vec_spb(nrhs, Ns) * nrhs * Ns;
  const int nb = vec_nblocks(h, nrhs, Ns);
  if (nblocks_out) *nblocks_out = nb;
  ODWF_PREC_SWITCH(prec, vec_norm2_kernel, dim3(nb), dim3(block), 0, st, v, sc, partial, h, nrhs, Ns);
  return hipGetLastError();
}

// copy right-hand side r_src of an nrhs_src field into right-hand side r_dst
// of an nrhs_dst field (same parity, any storage precisions); src == nullptr
// writes zeros
template <class PS, class PD>
__global__ void vec_copy_rhs_kernel(const void* src, const float* src_sc, int nrhs_src, int r_src,
                                    void* dst, float* dst_sc, int nrhs_dst, int r_dst, long h, int Ns) {
  using RS = typename PS::real;
  using RD = typename PD::real;
  const long n = h * Ns;
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
    const long j = k / Ns;
    const int s = (int)(k % Ns);
    cpx<RD> b[12];
    if (src) {
      cpx<RS> a[12];
      load_site<PS>(src, src_sc, j, r_src, s, nrhs_src, Ns, a);
#pragma unroll
      for (int c = 0; c < 12; c++) b[c] = {(RD)a[c].re, (RD)a[c].im};
    } else {
#pragma unroll
      for (int c = 0; c < 12; c++) b[c] = {RD(0), RD(0)};
    }
    store_site<PD>(dst, dst_sc, j, r_dst, s, nrhs_dst, Ns, b);
  }
}

template <class PS>
static hipError_t copy_rhs_to(int prec_dst, const void* src, const float* src_sc, int ns, int rs,
                              void* dst, float* dst_sc, int nd, int rd, long h, int Ns, hipStream_t st) {
  long nb = (h * Ns + 255) / 256;
  if (nb > 8192) nb = 8192;
  const dim3 gr((unsigned)nb);
  switch (prec_dst) {
    case PREC64: hipLaunchKernelGGL((vec_copy_rhs_kernel<PS, SP64>), gr, dim3(256), 0, st, src, src_sc, ns, rs, dst, dst_sc, nd, rd, h, Ns); break;
    case PREC32: hipLaunchKernelGGL((vec_copy_rhs_kernel<PS, SP32>), gr, dim3(256), 0, st, src, src_sc, ns, rs, dst, dst_sc, nd, rd, h, Ns); break;
    case PREC16: hipLaunchKernelGGL((vec_copy_rhs_kernel<PS, SP16>), gr, dim3(256), 0, st, src, src_sc, ns, rs, dst, dst_sc, nd, rd, h, Ns); break;
    case PRECB16: hipLaunchKernelGGL((vec_copy_rhs_kernel<PS, SPB16>), gr, dim3(256), 0, st, src, src_sc, ns, rs, dst, dst_sc, nd, rd, h, Ns); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_vec_copy_rhs(int prec_src, const void* src, const float* src_sc, int nrhs_src,
                               int r_src, int prec_dst, void* dst, float* dst_sc, int nrhs_dst,
                               int r_dst, long h, int Ns, hipStream_t st) {
  switch (prec_src) {
    case PREC64: return copy_rhs_to<SP64>(prec_dst, src, src_sc, nrhs_src, r_src, dst, dst_sc, nrhs_dst, r_dst, h, Ns, st);
    case PREC32: return copy_rhs_to<SP32>(prec_dst, src, src_sc, nrhs_src, r_src, dst, dst_sc, nrhs_dst, r_dst, h, Ns, st);
    case PREC16: return copy_rhs_to<SP16>(prec_dst, src, src_sc, nrhs_src, r_src, dst, dst_sc, nrhs_dst, r_dst, h, Ns, st);
    case PRECB16: return copy_rhs_to<SPB16>(prec_dst, src, src_sc, nrhs_src, r_src, dst, dst_sc, nrhs_dst, r_dst, h, Ns, st);
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// finalisation: one block of 256 threads
// ---------------------------------------------------------------------------
__global__ void fin_kernel(int kind, const double* partial, int nblocks, int nrhs, CGScal* scal,
                           double* out, int gated) {
  // all right-hand sides in one pass: thread t adds the partials of blocks
  // t, t + 256, ... per right-hand side, then one fixed tree over the threads
  __shared__ double red[MAXRHS * 256];
  __shared__ double sums[MAXRHS];
  double acc[MAXRHS];
#pragma unroll
  for (int r = 0; r < MAXRHS; r++) acc[r] = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
#pragma unroll
    for (int r = 0; r < MAXRHS; r++)
      if (r < nrhs) acc[r] += partial[(long)b * nrhs + r];
  }
#pragma unroll
  for (int r = 0; r < MAXRHS; r++)
    if (r < nrhs) red[r * 256 + threadIdx.x] = acc[r];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      for (int r = 0; r < nrhs; r++) red[r * 256 + threadIdx.x] += red[r * 256 + threadIdx.x + w];
    }
    __syncthreads();
  }
  if ((int)threadIdx.x < nrhs) sums[threadIdx.x] = red[threadIdx.x * 256];
  __syncthreads();
  if ((int)threadIdx.x >= nrhs) return;
  const int r = threadIdx.x;
  const double v = sums[r];
  if (out) out[r] = v;
  if (!scal) return;
  CGScal c = scal[r];
  if (gated && !c.update) return;  // only the right-hand sides that asked for it
  const bool finite = isfinite(v);
  switch (kind) {
    case FIN_F2:
      c.f2 = v;
      break;
    case FIN_ALPHA:
      c.pAp = v;
      if (c.active) {
        if (!finite || !(v > 0.0)) {
          c.nan = !finite;
          c.active = 0;
          c.alpha = 0.0;
        } else {
          c.alpha = c.rr / v;
        }
      } else {
        c.alpha = 0.0;
      }
      break;
    case FIN_BETA:
      if (c.active) {
        c.iters += 1;
        if (!finite) {
          c.nan = 1;
          c.active = 0;
          c.beta = 0.0;
        } else {
          c.beta = v / c.rr;
          c.rr = v;
          if (v > c.rmax2) c.rmax2 = v;
          const bool met = v <= c.tol2 * c.f2;
          const bool capped = c.iters >= c.maxiter;
          if (c.confirm) {
            // the decision is left to the true residual of the update that follows
            if (met || capped) c.update = 1;
            if (capped) c.active = 0;
          } else if (met) {
            c.converged = 1;
            c.active = 0;
          } else if (capped) {
            c.active = 0;
          }
          if (c.delta2 > 0.0 && v < c.delta2 * c.rmax2) c.update = 1;
        }
      } else {
        c.beta = 0.0;
      }
      break;
    case FIN_INIT:
      // v = |r|^2 of a freshly computed true residual
      c.rr = v;
      c.rmax2 = v;
      c.update = 0;
      if (c.iters > c.upd_iters) {  // an update of this right-hand side's own iterate
        c.nupd += 1;
        c.upd_iters = c.iters;
      }
      if (!finite) {
        c.nan = 1;
        c.active = 0;
      } else if (v <= c.tol2 * c.f2) {
        c.converged = 1;
        c.active = 0;
      } else {
        c.converged = 0;
        c.active = c.iters < c.maxiter ? 1 : 0;
      }
      break;
    default:
      break;
  }
  scal[r] = c;
}

// first stage of the finalisation for long partial arrays: block b sums the
// partials of blocks [b * 1024, (b + 1) * 1024) per right-hand side in a fixed
// tree and writes them to dst[b * nrhs + r]
__global__ void partial_reduce_kernel(const double* partial, int nblocks, int nrhs, double* dst) {
  __shared__ double red[MAXRHS * 256];
  const int b0 = blockIdx.x * 1024;
  const int b1 = min(b0 + 1024, nblocks);
  double acc[MAXRHS];
#pragma unroll
  for (int r = 0; r < MAXRHS; r++) acc[r] = 0.0;
  for (int b = b0 + threadIdx.x; b < b1; b += blockDim.x) {
#pragma unroll
    for (int r = 0; r < MAXRHS; r++)
      if (r < nrhs) acc[r] += partial[(long)b * nrhs + r];
  }
#pragma unroll
  for (int r = 0; r < MAXRHS; r++)
    if (r < nrhs) red[r * 256 + threadIdx.x] = acc[r];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      for (int r = 0; r < nrhs; r++) red[r * 256 + threadIdx.x] += red[r * 256 + threadIdx.x + w];
    }
    __syncthreads();
  }
  if ((int)threadIdx.x < nrhs) dst[(long)blockIdx.x * nrhs + threadIdx.x] = red[threadIdx.x * 256];
}

size_t partial_bytes(int nblocks, int nrhs) {
  return ((size_t)nblocks + (nblocks + 1023) / 1024 + 16) * nrhs * sizeof(double);
}

hipError_t launch_fin(int kind, const double* partial, int nblocks, int nrhs, CGScal* scal,
                      double* out, hipStream_t st, int gated) {
  if (nblocks > 2048) {
    // two stages; the second-stage inputs live behind the first-stage partials
    double* dst = const_cast<double*>(partial) + (size_t)nblocks * nrhs;
    const int nb2 = (nblocks + 1023) / 1024;
    hipLaunchKernelGGL(partial_reduce_kernel, dim3(nb2), dim3(256), 0, st, partial, nblocks, nrhs, dst);
    partial = dst;
    nblocks = nb2;
  }
  hipLaunchKernelGGL(fin_kernel, dim3(1), dim3(256), 0, st, kind, partial, nblocks, nrhs, scal, out,
                     gated);
  return hipGetLastError();
}

}  // namespace odwf
