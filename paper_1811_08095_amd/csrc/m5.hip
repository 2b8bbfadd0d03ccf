// Stand-alone fifth-dimension kernel on a half field:
//     out = c0 * prog(in) + c1 * other
// used for source preparation and reconstruction of the even-odd solve
// (omega^{-1}, A^{-1}, (1 + L)^{-1}, ...) and for the M5INV operator.  Sites are
// loaded in the lane layout (coalesced), transposed through LDS into columns of
// Ns values, transformed, and written back.
#include "dev_common.h"
#include "kernels.h"

namespace odwf {

template <class P, int NS>
__global__ void __launch_bounds__(256) m5_kernel(const void* in, const float* in_sc, void* out,
                                                 float* out_sc, const void* other,
                                                 const float* other_sc, double c0, double c1,
                                                 M5Prog prog, const void* coefp,
                                                 const KappaArr kappa, long h, int nrhs, int spb) {
  using R = typename P::real;
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NSP = NS + 1;
  const int inner = nrhs * NS;
  const int tid = threadIdx.x;
  const int sl = tid / inner, lr = tid - sl * inner, r = lr / NS, s = lr - r * NS;
  const long j0 = (long)blockIdx.x * spb;
  const int nsb = (int)min((long)spb, h - j0);
  const bool valid = sl < nsb;
  const long j = j0 + sl;
  cpx<R>* buf = reinterpret_cast<cpx<R>*>(smem);
  R* kap = reinterpret_cast<R*>(smem + (size_t)spb * nrhs * 12 * NSP * sizeof(cpx<R>));
  if (tid < nrhs) kap[tid] = (R)kappa.v[tid];

  cpx<R> v[12];
  if (valid) {
    load_site<P>(in, in_sc, j, r, s, nrhs, NS, v);
    cpx<R>* b = buf + ((size_t)(sl * nrhs + r) * 12) * NSP + s;
#pragma unroll
    for (int c = 0; c < 12; c++) b[c * NSP] = v[c];
  }
  __syncthreads();
  column_pass_lds<R, NS>(buf, nsb, nrhs, prog, reinterpret_cast<const R*>(coefp), kap);
  __syncthreads();
  if (!valid) return;
  const cpx<R>* b = buf + ((size_t)(sl * nrhs + r) * 12) * NSP + s;
#pragma unroll
  for (int c = 0; c < 12; c++) v[c] = cscale((R)c0, b[c * NSP]);
  if (other) {
    cpx<R> o[12];
    load_site<P>(other, other_sc, j, r, s, nrhs, NS, o);
#pragma unroll
    for (int c = 0; c < 12; c++) v[c] = cadd(v[c], cscale((R)c1, o[c]));
  }
  store_site<P>(out, out_sc, j, r, s, nrhs, NS, v);
}

template <class P, int NS>
static hipError_t launch_m5_t(const void* in, const float* in_sc, void* out, float* out_sc,
                              const void* other, const float* other_sc, double c0, double c1,
                              const M5Prog& prog, const void* coef, const KappaArr& kappa, long h,
                              int nrhs, hipStream_t st) {
  using R = typename P::real;
  const int inner = nrhs * NS;
  if (inner > 256 || nrhs > MAXRHS) return hipErrorInvalidValue;
  const int spb = 256 / inner;
  const int block = (spb * inner + 63) & ~63;
  const long nb = (h + spb - 1) / spb;
  const size_t sm = (size_t)spb * nrhs * 12 * (NS + 1) * sizeof(cpx<R>) + MAXRHS * sizeof(R);
  hipLaunchKernelGGL((m5_kernel<P, NS>), dim3((unsigned)nb), dim3(block), sm, st, in, in_sc, out,
                     out_sc, other, other_sc, c0, c1, prog, coef, kappa, h, nrhs, spb);
  return hipGetLastError();
}

template <class P>
static hipError_t launch_m5_p(const void* in, const float* in_sc, void* out, float* out_sc,
                              const void* other, const float* other_sc, double c0, double c1,
                              const M5Prog& prog, const void* coef, const KappaArr& kappa, long h,
                              int nrhs, int Ns, hipStream_t st) {
  switch (Ns) {
    case 4: return launch_m5_t<P, 4>(in, in_sc, out, out_sc, other, other_sc, c0, c1, prog, coef, kappa, h, nrhs, st);
    case 8: return launch_m5_t<P, 8>(in, in_sc, out, out_sc, other, other_sc, c0, c1, prog, coef, kappa, h, nrhs, st);
    case 16: return launch_m5_t<P, 16>(in, in_sc, out, out_sc, other, other_sc, c0, c1, prog, coef, kappa, h, nrhs, st);
    case 32: return launch_m5_t<P, 32>(in, in_sc, out, out_sc, other, other_sc, c0, c1, prog, coef, kappa, h, nrhs, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_m5(int prec, const void* in, const float* in_sc, void* out, float* out_sc,
                     const void* other, const float* other_sc, double c0, double c1,
                     const M5Prog& prog, const void* coef, const KappaArr& kappa, long h, int nrhs,
                     int Ns, hipStream_t st) {
  switch (prec) {
    case PREC64: return launch_m5_p<SP64>(in, in_sc, out, out_sc, other, other_sc, c0, c1, prog, coef, kappa, h, nrhs, Ns, st);
    case PREC32: return launch_m5_p<SP32>(in, in_sc, out, out_sc, other, other_sc, c0, c1, prog, coef, kappa, h, nrhs, Ns, st);
    case PREC16: return launch_m5_p<SP16>(in, in_sc, out, out_sc, other, other_sc, c0, c1, prog, coef, kappa, h, nrhs, Ns, st);
    case PRECB16: return launch_m5_p<SPB16>(in, in_sc, out, out_sc, other, other_sc, c0, c1, prog, coef, kappa, h, nrhs, Ns, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace odwf
