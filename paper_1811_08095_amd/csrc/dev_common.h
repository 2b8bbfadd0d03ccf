// Device-side building blocks shared by the HIP kernels of libodwf:
// complex arithmetic, spinor storage policies (FP64 / FP32 / FP16+scale /
// BF16+scale), link formats, fifth-dimension programs and deterministic
// per-right-hand-side block reductions.
//
// Internal spinor layout of one parity half (h = V/2 sites), per site j,
// right-hand side r, fifth-dimension slice s and spin-colour component
// c = spin*3 + colour (12 complex per 5D site):
//     chunk (j, r, cg, s) of CPB consecutive complex numbers, cg = c / CPB,
//     address = ((j * nrhs + r) * NCG + cg) * Ns + s   (in 16-byte chunks),
// so the Ns lanes of one (site, rhs) read consecutive 16-byte chunks and the
// chunk stride within a 5D site is the compile-time Ns.  The
// reduced-precision formats keep one float scale per 5D site (j, r, s) at
// (j * nrhs + r) * Ns + s; stored values are component / scale with scale the
// largest |real| or |imag| part of the 24 reals.
#pragma once
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "odwf_types.h"

namespace odwf {

template <class R>
struct cpx {
  R re, im;
};

template <class R>
__device__ __forceinline__ cpx<R> cadd(cpx<R> a, cpx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <class R>
__device__ __forceinline__ cpx<R> csub(cpx<R> a, cpx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <class R>
__device__ __forceinline__ cpx<R> cscale(R f, cpx<R> a) { return {f * a.re, f * a.im}; }
// a * b
template <class R>
__device__ __forceinline__ cpx<R> cmul(cpx<R> a, cpx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// acc + a * b
template <class R>
__device__ __forceinline__ cpx<R> cfma(cpx<R> a, cpx<R> b, cpx<R> acc) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
  return acc;
}
// i * a
template <class R>
__device__ __forceinline__ cpx<R> cmuli(cpx<R> a) { return {-a.im, a.re}; }
template <class R>
__device__ __forceinline__ R cnorm2(cpx<R> a) { return a.re * a.re + a.im * a.im; }

// ---------------------------------------------------------------------------
// storage policies
// ---------------------------------------------------------------------------

struct SP64 {
  using real = double;
  static constexpr int CPB = 1;  // complex per 16-byte chunk
  static constexpr bool SCALED = false;
  static constexpr int BYTES = 16;  // bytes per complex
};
struct SP32 {
  using real = float;
  static constexpr int CPB = 2;
  static constexpr bool SCALED = false;
  static constexpr int BYTES = 8;
};
struct SP16 {
  using real = float;
  static constexpr int CPB = 4;
  static constexpr bool SCALED = true;
  static constexpr int BYTES = 4;
};
struct SPB16 {
  using real = float;
  static constexpr int CPB = 4;
  static constexpr bool SCALED = true;
  static constexpr int BYTES = 4;
};

// BF16 stores through the hardware conversion (1, default) or the integer
// rounding of f_to_bf16 (0); both round to nearest even
#ifndef ODWF_HW_BF16_CVT
#define ODWF_HW_BF16_CVT 1
#endif
__device__ __forceinline__ float bf16_to_f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }
__device__ __forceinline__ uint16_t f_to_bf16(float f) {
  // round to nearest even; inputs are finite and bounded by 1 after scaling
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// unpack one 16-byte chunk into CPB complex values
template <class P>
__device__ __forceinline__ void unpack_chunk(const uint4 q, cpx<typename P::real>* v);

template <>
__device__ __forceinline__ void unpack_chunk<SP64>(const uint4 q, cpx<double>* v) {
  v[0].re = __hiloint2double((int)q.y, (int)q.x);
  v[0].im = __hiloint2double((int)q.w, (int)q.z);
}
template <>
__device__ __forceinline__ void unpack_chunk<SP32>(const uint4 q, cpx<float>* v) {
  v[0] = {__uint_as_float(q.x), __uint_as_float(q.y)};
  v[1] = {__uint_as_float(q.z), __uint_as_float(q.w)};
}
template <>
__device__ __forceinline__ void unpack_chunk<SP16>(const uint4 q, cpx<float>* v) {
  const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
  for (int k = 0; k < 4; k++) {
    __half2 hh = *reinterpret_cast<const __half2*>(&w[k]);
    float2 f = __half22float2(hh);
    v[k] = {f.x, f.y};
  }
}
template <>
__device__ __forceinline__ void unpack_chunk<SPB16>(const uint4 q, cpx<float>* v) {
  const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
  for (int k = 0; k < 4; k++) v[k] = {bf16_to_f((uint16_t)(w[k] & 0xffffu)), bf16_to_f((uint16_t)(w[k] >> 16))};
}

template <class P>
__device__ __forceinline__ uint4 pack_chunk(const cpx<typename P::real>* v, typename P::real inv);

template <>
__device__ __forceinline__ uint4 pack_chunk<SP64>(const cpx<double>* v, double) {
  uint4 q;
  q.x = (uint32_t)__double2loint(v[0].re);
  q.y = (uint32_t)__double2hiint(v[0].re);
  q.z = (uint32_t)__double2loint(v[0].im);
  q.w = (uint32_t)__double2hiint(v[0].im);
  return q;
}
template <>
__device__ __forceinline__ uint4 pack_chunk<SP32>(const cpx<float>* v, float) {
  return make_uint4(__float_as_uint(v[0].re), __float_as_uint(v[0].im), __float_as_uint(v[1].re),
                    __float_as_uint(v[1].im));
}
template <>
__device__ __forceinline__ uint4 pack_chunk<SP16>(const cpx<float>* v, float inv) {
  uint32_t w[4];
#pragma unroll
  for (int k = 0; k < 4; k++) {
    __half2 hh = __floats2half2_rn(v[k].re * inv, v[k].im * inv);
    w[k] = *reinterpret_cast<uint32_t*>(&hh);
  }
  return make_uint4(w[0], w[1], w[2], w[3]);
}
template <>
__device__ __forceinline__ uint4 pack_chunk<SPB16>(const cpx<float>* v, float inv) {
  uint32_t w[4];
#pragma unroll
  for (int k = 0; k < 4; k++) {
#if ODWF_HW_BF16_CVT
    // one v_cvt_pk_bf16_f32 per complex (gfx950): round to nearest even, as f_to_bf16
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    const f32x2 f = {v[k].re * inv, v[k].im * inv};
    w[k] = __builtin_bit_cast(uint32_t, __builtin_convertvector(f, bf16x2));
#else
    w[k] = (uint32_t)f_to_bf16(v[k].re * inv) | ((uint32_t)f_to_bf16(v[k].im * inv) << 16);
#endif
  }
  return make_uint4(w[0], w[1], w[2], w[3]);
}

// Spinor half-field view
template <class P>
struct HalfView {
  const uint4* __restrict__ base;
  const float* __restrict__ scale;
};

// load the 12 components of 5D site (j, r, s); NT = 1: nontemporal loads
// (a stream read once, which should not displace re-used rows from L2)
template <class P, int NT = 0>
__device__ __forceinline__ void load_site(const void* base, const float* scale, long j, int r, int s,
                                          int nrhs, int Ns, cpx<typename P::real> (&v)[12]) {
  constexpr int NCG = 12 / P::CPB;
  const uint4* b = reinterpret_cast<const uint4*>(base);
  const long off = ((j * nrhs + r) * NCG) * Ns + s;
  uint4 q[NCG];
#pragma unroll
  for (int cg = 0; cg < NCG; cg++) {
    if constexpr (NT) {
      typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
      const u32x4 w = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(b + off + cg * Ns));
      q[cg] = make_uint4(w.x, w.y, w.z, w.w);
    } else {
      q[cg] = b[off + cg * Ns];
    }
  }
#pragma unroll
  for (int cg = 0; cg < NCG; cg++) unpack_chunk<P>(q[cg], &v[cg * P::CPB]);
  if constexpr (P::SCALED) {
    float sc = scale[(j * nrhs + r) * Ns + s];
#pragma unroll
    for (int c = 0; c < 12; c++) v[c] = cscale(sc, v[c]);
  }
}

// cached variant: for neighbour reads that other sites re-use
template <class P>
__device__ __forceinline__ void load_site_cached(const void* base, const float* scale, long j, int r,
                                                 int s, int nrhs, int Ns,
                                                 cpx<typename P::real> (&v)[12]) {
  constexpr int NCG = 12 / P::CPB;
  const uint4* b = reinterpret_cast<const uint4*>(base);
  const long off = ((j * nrhs + r) * NCG) * Ns + s;
  uint4 q[NCG];
#pragma unroll
  for (int cg = 0; cg < NCG; cg++) q[cg] = b[off + cg * Ns];
#pragma unroll
  for (int cg = 0; cg < NCG; cg++) unpack_chunk<P>(q[cg], &v[cg * P::CPB]);
  if constexpr (P::SCALED) {
    float sc = scale[(j * nrhs + r) * Ns + s];
#pragma unroll
    for (int c = 0; c < 12; c++) v[c] = cscale(sc, v[c]);
  }
}

// cached neighbour read without the per-site scale applied: v holds the
// stored values, *sc the site's scale (1 for unscaled formats), so that the
// caller can apply the scale after its linear algebra on fewer numbers
template <class P>
__device__ __forceinline__ void load_site_cached_raw(const void* base, const float* scale, long j,
                                                     int r, int s, int nrhs, int Ns,
                                                     cpx<typename P::real> (&v)[12],
                                                     typename P::real& sc) {
  constexpr int NCG = 12 / P::CPB;
  const uint4* b = reinterpret_cast<const uint4*>(base);
  const long off = ((j * nrhs + r) * NCG) * Ns + s;
  uint4 q[NCG];
#pragma unroll
  for (int cg = 0; cg < NCG; cg++) q[cg] = b[off + cg * Ns];
#pragma unroll
  for (int cg = 0; cg < NCG; cg++) unpack_chunk<P>(q[cg], &v[cg * P::CPB]);
  if constexpr (P::SCALED) sc = scale[(j * nrhs + r) * Ns + s];
  else sc = typename P::real(1);
}

// NT = 1: nontemporal stores (written once, not re-read by this launch)
#ifndef ODWF_NT_STORE
#define ODWF_NT_STORE 0
#endif
#ifndef ODWF_NT_LINKS
#define ODWF_NT_LINKS 0
#endif
template <class P, int NT = 0>
__device__ __forceinline__ void store_site(void* base, float* scale, long j, int r, int s, int nrhs,
                                           int Ns, const cpx<typename P::real> (&v)[12]) {
  using R = typename P::real;
  constexpr int NCG = 12 / P::CPB;
  uint4* b = reinterpret_cast<uint4*>(base);
  const long off = ((j * nrhs + r) * NCG) * Ns + s;
  R inv = R(1);
  if constexpr (P::SCALED) {
    float m = 0.f;
#pragma unroll
    for (int c = 0; c < 12; c++) m = fmaxf(m, fmaxf(fabsf(v[c].re), fabsf(v[c].im)));
    if constexpr (NT) __builtin_nontemporal_store(m, scale + (j * nrhs + r) * Ns + s);
    else scale[(j * nrhs + r) * Ns + s] = m;
    inv = m > 0.f ? 1.0f / m : 0.f;
  }
#pragma unroll
  for (int cg = 0; cg < NCG; cg++) {
    const uint4 q = pack_chunk<P>(&v[cg * P::CPB], inv);
    if constexpr (NT) {
      typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
      const u32x4 w = {q.x, q.y, q.z, q.w};
      __builtin_nontemporal_store(w, reinterpret_cast<u32x4*>(b + off + cg * Ns));
    } else {
      b[off + cg * Ns] = q;
    }
  }
}

// ---------------------------------------------------------------------------
// spin projection in the chiral basis (shared by the hopping and force kernels)
// ---------------------------------------------------------------------------

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

// is right-hand side r selected by the gate?
__device__ __forceinline__ bool gate_on(const CGScal* g, int mode, int r) {
  if (!g || mode == GATE_NONE) return true;
  return mode == GATE_ACTIVE ? g[r].active != 0 : g[r].update != 0;
}
// does any right-hand side of the launch pass the gate? (block-uniform)
__device__ __forceinline__ bool gate_any(const CGScal* g, int mode, int nrhs) {
  if (!g || mode == GATE_NONE) return true;
  bool any = false;
  for (int r = 0; r < nrhs; r++) any |= gate_on(g, mode, r);
  return any;
}

// ---------------------------------------------------------------------------
// fifth-dimension programs on one column y[0..NS-1] (one 4D site, one
// right-hand side, one spin-colour component), in the chirality-local order:
// chirality + (spins 0, 1) uses s as is, chirality - (spins 2, 3) uses the
// mirrored index NS-1-s, in which L_- takes the same lower-shift form as L_+.
// ---------------------------------------------------------------------------

// coefficient table coef[chi][id][s] in global memory; the column passes
// make chi wave-uniform so the coefficients come in through scalar loads
template <class R, int NS>
__device__ __forceinline__ void m5_run(const M5Prog& prog, cpx<R> (&y)[NS], const R* __restrict__ cf,
                                       R kappa) {
  for (int k = 0; k < prog.n; k++) {
    const M5Op op = prog.op[k];
    const R* d = cf + op.d * NS;
    const R* e = cf + op.e * NS;
    switch (op.type) {
      case M5_SCALE: {
#pragma unroll
        for (int s = 0; s < NS; s++) y[s] = cscale(d[s], y[s]);
      } break;
      case M5_MUL_LO: {  // z_s = d_s y_s + e_s y_{s-1};  z_0 = d_0 y_0 + kappa e_0 y_{NS-1}
        cpx<R> last = y[NS - 1];
#pragma unroll
        for (int s = NS - 1; s >= 1; s--) y[s] = cadd(cscale(d[s], y[s]), cscale(e[s], y[s - 1]));
        y[0] = cadd(cscale(d[0], y[0]), cscale(kappa * e[0], last));
      } break;
      case M5_MUL_UP: {  // z_s = d_s y_s + e_s y_{s+1};  z_{NS-1} = d y + kappa e_{NS-1} y_0
        cpx<R> first = y[0];
#pragma unroll
        for (int s = 0; s < NS - 1; s++) y[s] = cadd(cscale(d[s], y[s]), cscale(e[s], y[s + 1]));
        y[NS - 1] = cadd(cscale(d[NS - 1], y[NS - 1]), cscale(kappa * e[NS - 1], first));
      } break;
      case M5_SOLVE_LO: {  // inverse of MUL_LO; d holds 1/d
        // y_s = p_s + q_s y_{N-1}; p by forward substitution, q recomputed
        R q = -kappa * e[0] * d[0];
        y[0] = cscale(d[0], y[0]);
#pragma unroll
        for (int s = 1; s < NS; s++) {
          q = -e[s] * q * d[s];
          y[s] = cscale(d[s], csub(y[s], cscale(e[s], y[s - 1])));
        }
        const cpx<R> vl = cscale(R(1) / (R(1) - q), y[NS - 1]);
        y[NS - 1] = vl;
        q = -kappa * e[0] * d[0];
#pragma unroll
        for (int s = 0; s < NS - 1; s++) {
          if (s > 0) q = -e[s] * q * d[s];
          y[s] = cadd(y[s], cscale(q, vl));
        }
      } break;
      case M5_SOLVE_UP: {  // inverse of MUL_UP; d holds 1/d
        R q = -kappa * e[NS - 1] * d[NS - 1];
        y[NS - 1] = cscale(d[NS - 1], y[NS - 1]);
#pragma unroll
        for (int s = NS - 2; s >= 0; s--) {
          q = -e[s] * q * d[s];
          y[s] = cscale(d[s], csub(y[s], cscale(e[s], y[s + 1])));
        }
        const cpx<R> v0 = cscale(R(1) / (R(1) - q), y[0]);
        y[0] = v0;
        q = -kappa * e[NS - 1] * d[NS - 1];
#pragma unroll
        for (int s = NS - 1; s >= 1; s--) {
          if (s < NS - 1) q = -e[s] * q * d[s];
          y[s] = cadd(y[s], cscale(q, v0));
        }
      } break;
      default: break;
    }
  }
}

// the same programs applied in place to one LDS column (element s at
// col[chi ? NS - 1 - s : s]), streaming through it with O(1) registers
template <class R, int NS>
__device__ __forceinline__ void m5_run_lds(const M5Prog& prog, cpx<R>* col, int chi,
                                           const R* __restrict__ cf, R kappa) {
  const int st = chi ? -1 : 1;
  cpx<R>* c0 = col + (chi ? NS - 1 : 0);  // element s at c0[s * st]
  for (int k = 0; k < prog.n; k++) {
    const M5Op op = prog.op[k];
    const R* d = cf + op.d * NS;
    const R* e = cf + op.e * NS;
    switch (op.type) {
      case M5_SCALE: {
#pragma unroll 4
        for (int s = 0; s < NS; s++) c0[s * st] = cscale(d[s], c0[s * st]);
      } break;
      case M5_MUL_LO: {
        const cpx<R> last = c0[(NS - 1) * st];
        cpx<R> hi = last;
#pragma unroll 4
        for (int s = NS - 1; s >= 1; s--) {
          const cpx<R> lo = c0[(s - 1) * st];
          c0[s * st] = cadd(cscale(d[s], hi), cscale(e[s], lo));
          hi = lo;
        }
        c0[0] = cadd(cscale(d[0], hi), cscale(kappa * e[0], last));
      } break;
      case M5_MUL_UP: {
        const cpx<R> first = c0[0];
        cpx<R> lo = first;
#pragma unroll 4
        for (int s = 0; s < NS - 1; s++) {
          const cpx<R> hi = c0[(s + 1) * st];
          c0[s * st] = cadd(cscale(d[s], lo), cscale(e[s], hi));
          lo = hi;
        }
        c0[(NS - 1) * st] = cadd(cscale(d[NS - 1], lo), cscale(kappa * e[NS - 1], first));
      } break;
      case M5_SOLVE_LO: {
        R q = -kappa * e[0] * d[0];
        cpx<R> prev = cscale(d[0], c0[0]);
        c0[0] = prev;
#pragma unroll 4
        for (int s = 1; s < NS; s++) {
          q = -e[s] * q * d[s];
          prev = cscale(d[s], csub(c0[s * st], cscale(e[s], prev)));
          c0[s * st] = prev;
        }
        const cpx<R> vl = cscale(R(1) / (R(1) - q), prev);
        c0[(NS - 1) * st] = vl;
        q = -kappa * e[0] * d[0];
#pragma unroll 4
        for (int s = 0; s < NS - 1; s++) {
          if (s > 0) q = -e[s] * q * d[s];
          c0[s * st] = cadd(c0[s * st], cscale(q, vl));
        }
      } break;
      case M5_SOLVE_UP: {
        R q = -kappa * e[NS - 1] * d[NS - 1];
        cpx<R> prev = cscale(d[NS - 1], c0[(NS - 1) * st]);
        c0[(NS - 1) * st] = prev;
#pragma unroll 4
        for (int s = NS - 2; s >= 0; s--) {
          q = -e[s] * q * d[s];
          prev = cscale(d[s], csub(c0[s * st], cscale(e[s], prev)));
          c0[s * st] = prev;
        }
        const cpx<R> v0 = cscale(R(1) / (R(1) - q), prev);
        c0[0] = v0;
        q = -kappa * e[NS - 1] * d[NS - 1];
#pragma unroll 4
        for (int s = NS - 1; s >= 1; s--) {
          if (s < NS - 1) q = -e[s] * q * d[s];
          c0[s * st] = cadd(c0[s * st], cscale(q, v0));
        }
      } break;
      default: break;
    }
  }
}

// ---------------------------------------------------------------------------
// the same programs with the column spread over lanes: for N_s = 16 the 16
// slices of one (site, right-hand side) are the 16 lanes of one DPP row, so
// every lane keeps its own slice of all 12 components in registers and the
// fifth-dimension couplings become cross-lane moves inside the row.  The
// bidiagonal products need the neighbouring slice (a row rotation); the cyclic
// bidiagonal solves are first-order linear recurrences x_u = a_u x_{u-1} + b_u,
// solved by a log2(16)-step scan over the affine maps (a, b), closed around the
// cycle with x_last = b_last / (1 - a_last) and one broadcast in the row.
// FP32 arithmetic only; chirality + runs in slice order, chirality - in the
// mirrored order (as in m5_run).
// ---------------------------------------------------------------------------
#ifndef ODWF_LANE_PASS
#define ODWF_LANE_PASS 1
#endif
template <class R, int NS>
struct LanePass {
  static constexpr bool on = ODWF_LANE_PASS && sizeof(R) == 4 && NS == 16;
};

// DPP16 row controls: lane i reads lane i - n (SHR), i + n (SHL), (i - n) mod 16
// (ROR) or lane n of its row (NEWBCAST, gfx90a and later)
constexpr int DPP_SHL(int n) { return 0x100 + n; }
constexpr int DPP_SHR(int n) { return 0x110 + n; }
constexpr int DPP_ROR(int n) { return 0x120 + n; }
constexpr int DPP_NEWBCAST(int n) { return 0x150 + n; }

// value of v in the lane given by CTRL; lanes whose source lies outside the
// row read 0 (bound_ctrl), so no register has to be preset with an old value
template <int CTRL>
__device__ __forceinline__ float row_move0(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
// the same with a chosen value `old` for lanes whose source lies outside the row
template <int CTRL>
__device__ __forceinline__ float row_move(float old, float v) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), CTRL, 0xF, 0xF, false));
}
// value of v in lane 15 (LAST) or lane 0 of the lane's row: a DPP row
// broadcast, no trip through the LDS crossbar
template <bool LAST>
__device__ __forceinline__ float row_bcast(float v) {
  return row_move0<DPP_NEWBCAST(LAST ? 15 : 0)>(v);
}

// y[c0 .. c0+5] = d y + e y_nb, with y_nb the value of the neighbouring slice
template <int CTRL>
__device__ __forceinline__ void lane_mul(cpx<float> (&y)[12], int c0, float d, float e) {
#pragma unroll
  for (int c = c0; c < c0 + 6; c++) {
    const float nr = row_move0<CTRL>(y[c].re), ni = row_move0<CTRL>(y[c].im);
    y[c] = {d * y[c].re + e * nr, d * y[c].im + e * ni};
  }
}

// y[c0 .. c0+5] <- solution of x_u = a x_{u-1} + b_u (b_u = y on entry) around
// the cycle; DOWN: element u - 1 sits in the next lower lane (else the next
// higher one); LAST: the final element in scan order sits in lane 15 (else 0)
template <bool DOWN, bool LAST>
__device__ __forceinline__ void lane_solve(cpx<float> (&y)[12], int c0, float a) {
#pragma unroll
  for (int k = 1; k < 16; k <<= 1) {
    float pa;
#pragma unroll
    for (int c = c0; c < c0 + 6; c++) {
      float pr, pi;
      // lanes before the start of the scan read 0: their term vanishes
      if (k == 1) {
        pr = DOWN ? row_move0<DPP_SHR(1)>(y[c].re) : row_move0<DPP_SHL(1)>(y[c].re);
        pi = DOWN ? row_move0<DPP_SHR(1)>(y[c].im) : row_move0<DPP_SHL(1)>(y[c].im);
      } else if (k == 2) {
        pr = DOWN ? row_move0<DPP_SHR(2)>(y[c].re) : row_move0<DPP_SHL(2)>(y[c].re);
        pi = DOWN ? row_move0<DPP_SHR(2)>(y[c].im) : row_move0<DPP_SHL(2)>(y[c].im);
      } else if (k == 4) {
        pr = DOWN ? row_move0<DPP_SHR(4)>(y[c].re) : row_move0<DPP_SHL(4)>(y[c].re);
        pi = DOWN ? row_move0<DPP_SHR(4)>(y[c].im) : row_move0<DPP_SHL(4)>(y[c].im);
      } else {
        pr = DOWN ? row_move0<DPP_SHR(8)>(y[c].re) : row_move0<DPP_SHL(8)>(y[c].re);
        pi = DOWN ? row_move0<DPP_SHR(8)>(y[c].im) : row_move0<DPP_SHL(8)>(y[c].im);
      }
      y[c] = {y[c].re + a * pr, y[c].im + a * pi};
    }
    if (k == 1) pa = DOWN ? row_move<DPP_SHR(1)>(1.f, a) : row_move<DPP_SHL(1)>(1.f, a);
    else if (k == 2) pa = DOWN ? row_move<DPP_SHR(2)>(1.f, a) : row_move<DPP_SHL(2)>(1.f, a);
    else if (k == 4) pa = DOWN ? row_move<DPP_SHR(4)>(1.f, a) : row_move<DPP_SHL(4)>(1.f, a);
    else pa = DOWN ? row_move<DPP_SHR(8)>(1.f, a) : row_move<DPP_SHL(8)>(1.f, a);
    a *= pa;
  }
  // a is now the product of the step factors up to this lane; close the cycle
  const float g = 1.f / (1.f - a);
#pragma unroll
  for (int c = c0; c < c0 + 6; c++) {
    const float xr = row_bcast<LAST>(g * y[c].re), xi = row_bcast<LAST>(g * y[c].im);
    y[c] = {y[c].re + a * xr, y[c].im + a * xi};
  }
}

// the program loop unrolled over its four op slots (1, default), so the
// coefficient reads of a step can be issued before the previous step ends
#ifndef ODWF_M5_UNROLL
#define ODWF_M5_UNROLL 1
#endif
template <int NS>
__device__ __forceinline__ void m5_run_lanes(const M5Prog& prog, cpx<float> (&y)[12],
                                             const float* __restrict__ cf, float kappa, int s) {
  static_assert(NS == 16, "one DPP row per column");
  const int up = s, um = NS - 1 - s;  // chirality-local slice index, chirality + and -
  const float* cfm = cf + NCOEF * NS;
#if ODWF_M5_UNROLL
#pragma unroll
  for (int k = 0; k < (int)(sizeof(prog.op) / sizeof(prog.op[0])); k++) {
    if (k >= prog.n) break;
#else
  for (int k = 0; k < prog.n; k++) {
#endif
    const M5Op op = prog.op[k];
    const float dp = cf[op.d * NS + up], dm = cfm[op.d * NS + um];
    float ep = cf[op.e * NS + up], em = cfm[op.e * NS + um];
    switch (op.type) {
      case M5_SCALE: {
#pragma unroll
        for (int c = 0; c < 12; c++) y[c] = cscale(c < 6 ? dp : dm, y[c]);
      } break;
      case M5_MUL_LO: {  // local u - 1: lane s - 1 (chirality +), s + 1 (chirality -)
        if (up == 0) ep *= kappa;
        if (um == 0) em *= kappa;
        lane_mul<DPP_ROR(1)>(y, 0, dp, ep);
        lane_mul<DPP_ROR(15)>(y, 6, dm, em);
      } break;
      case M5_MUL_UP: {  // local u + 1: lane s + 1 (chirality +), s - 1 (chirality -)
        if (up == NS - 1) ep *= kappa;
        if (um == NS - 1) em *= kappa;
        lane_mul<DPP_ROR(15)>(y, 0, dp, ep);
        lane_mul<DPP_ROR(1)>(y, 6, dm, em);
      } break;
      case M5_SOLVE_LO: {  // x_u = d_u (y_u - e_u x_{u-1}), x_{-1} = x_{N-1} with e_0 -> kappa e_0
        if (up == 0) ep *= kappa;
        if (um == 0) em *= kappa;
#pragma unroll
        for (int c = 0; c < 12; c++) y[c] = cscale(c < 6 ? dp : dm, y[c]);
        lane_solve<true, true>(y, 0, -dp * ep);    // chirality +: from lane s - 1, ends at lane 15
        lane_solve<false, false>(y, 6, -dm * em);  // chirality -: from lane s + 1, ends at lane 0
      } break;
      case M5_SOLVE_UP: {  // x_u = d_u (y_u - e_u x_{u+1}), x_N = x_0 with e_{N-1} -> kappa e_{N-1}
        if (up == NS - 1) ep *= kappa;
        if (um == NS - 1) em *= kappa;
#pragma unroll
        for (int c = 0; c < 12; c++) y[c] = cscale(c < 6 ? dp : dm, y[c]);
        lane_solve<false, false>(y, 0, -dp * ep);  // chirality +: from lane s + 1, ends at lane 0
        lane_solve<true, true>(y, 6, -dm * em);    // chirality -: from lane s - 1, ends at lane 15
      } break;
      default: break;
    }
  }
}

// ---------------------------------------------------------------------------
// column pass: buf holds [site][rhs][12 components][NS + 1] values; every
// column (site, rhs, component) of NS values is transformed by prog.  Items
// are ordered (chirality, site, rhs, component-of-chirality) with each
// chirality padded to a multiple of 64, so chirality is uniform per wave.
// blockDim.x must be a multiple of 64.  Caller synchronises around it.
// ---------------------------------------------------------------------------
template <class R, int NS>
__device__ __forceinline__ void column_pass_lds(cpx<R>* buf, int nsb, int nrhs, const M5Prog& prog,
                                                const R* coef, const R* kap) {
  constexpr int NSP = NS + 1;
  const int per = nsb * nrhs * 6;
  const int ipc = (per + 63) & ~63;
  const int lane = threadIdx.x & 63;
  for (int base = threadIdx.x & ~63; base < 2 * ipc; base += blockDim.x) {
    const int chi = __builtin_amdgcn_readfirstlane(base / ipc);
    const int q = base - chi * ipc + lane;
    if (q < per) {
      const int c6 = q % 6;
      const int sr = q / 6;  // sl * nrhs + r
      const int rr = sr % nrhs;
      cpx<R>* col = buf + ((size_t)sr * 12 + chi * 6 + c6) * NSP;
      if constexpr (sizeof(R) == 8) {
        // FP64: a column in registers (2 NS doubles per component) would cap the
        // fused hopping kernel at one wave per SIMD; streamed through LDS it
        // runs two (measured 5 % faster for the normal operator)
        m5_run_lds<R, NS>(prog, col, chi, coef + chi * NCOEF * NS, kap[rr]);
      } else {
        // FP32 arithmetic: the register column is faster than streaming
        cpx<R> yv[NS];
#pragma unroll
        for (int s = 0; s < NS; s++) yv[s] = col[chi ? NS - 1 - s : s];
        m5_run<R, NS>(prog, yv, coef + chi * NCOEF * NS, kap[rr]);
#pragma unroll
        for (int s = 0; s < NS; s++) col[chi ? NS - 1 - s : s] = yv[s];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// deterministic per-right-hand-side block reduction of one double per lane.
// Lanes are laid out (site slot sl, right-hand side r, slice s) with s fastest,
// tid = (sl * nrhs + r) * Ns + s (Ns a power of two dividing 64, so the Ns
// lanes of one (site, r) lie in one wave).  Those Ns lanes add their values by
// a fixed xor butterfly of cross-lane moves (no LDS traffic; every lane ends
// with the same bits, each pairwise addition being commutative); lane s = 0
// puts the sum in tmp[sl * nrhs + r]; one lane per right-hand side then adds
// the nsl site sums in site order and writes partial[slot * nrhs + r].
// All threads of the block call it; padded threads (g >= nsl * nrhs) pass 0.
// tmp: LDS of at least nsl * nrhs doubles.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void block_reduce_rhs(double v, int Ns, int nsl, int nrhs, double* tmp,
                                                 double* partial, long slot) {
  for (int m = Ns >> 1; m >= 1; m >>= 1) v += __shfl_xor(v, m, Ns);
  const int tid = threadIdx.x;
  const int g = tid / Ns;
  __syncthreads();  // tmp may alias LDS the block used before
  if ((tid & (Ns - 1)) == 0 && g < nsl * nrhs) tmp[g] = v;
  __syncthreads();
  if (tid < nrhs) {
    double acc = 0.0;
    for (int k = 0; k < nsl; k++) acc += tmp[k * nrhs + tid];
    partial[slot * nrhs + tid] = acc;
  }
}

}  // namespace odwf
