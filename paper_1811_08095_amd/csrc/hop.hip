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
// as products of cyclic bidiagonal factors), and optionally the fused CG
// residual step r -= alpha y with its |r|^2 partial sums.
//
// Thread layout: a block holds spb sites of the output parity; each site has
// nrhs * Ns lanes (s fastest) that read consecutive 16-byte chunks of every
// neighbour.  The 8 links of the block's sites are staged once in LDS and
// shared by all nrhs * Ns lanes of a site (links are stored per output parity
// as [site][8][...] with directions 0-3 forward U_mu(x) and 4-7 backward
// U_mu(x - mu)^dag).  Fifth-dimension programs run across the 16 lanes of a
// DPP row for FP32 arithmetic at Ns = 16 (one slice per lane), otherwise on LDS
// columns (site, r, colour-spin component) of Ns values.  No MFMA: the stencil
// is a string of 3x3 complex mat-vecs; its time is set by the traffic between
// the L2 caches and memory (FP32, FP64) or by VALU issue (FP16, BF16 storage).
#include <type_traits>

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

// stage the links of `nsb` sites starting at j0 into LDS as 9 complex per
// matrix, times -1/2 (the factor of the hopping term: a power of two, so the
// hop sums round exactly as with the factor applied at the end)
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
      lnk[q] = cscale(-0.5, z);
    }
  } else {
    const float4* src = reinterpret_cast<const float4*>(links) + j0 * 8 * 3;
    for (int m = threadIdx.x; m < nmat; m += blockDim.x) {
#if ODWF_NT_LINKS
      // links are read once per launch: keep them from displacing spinor rows in L2
      typedef float f32x4 __attribute__((ext_vector_type(4)));
      const f32x4* sv = reinterpret_cast<const f32x4*>(src + m * 3);
      const f32x4 av = __builtin_nontemporal_load(sv), bv = __builtin_nontemporal_load(sv + 1),
                  cv = __builtin_nontemporal_load(sv + 2);
      float4 a = make_float4(av.x, av.y, av.z, av.w), b = make_float4(bv.x, bv.y, bv.z, bv.w),
             c = make_float4(cv.x, cv.y, cv.z, cv.w);
#else
      float4 a = src[m * 3 + 0], b = src[m * 3 + 1], c = src[m * 3 + 2];
#endif
      cpx<float> u[6] = {{a.x, a.y}, {a.z, a.w}, {b.x, b.y}, {b.z, b.w}, {c.x, c.y}, {c.z, c.w}};
      cpx<R>* d = lnk + m * 9;
#pragma unroll
      for (int k = 0; k < 6; k++) d[k] = cscale(-0.5f, u[k]);
      // row2[a] = conj(row0[b] row1[c] - row0[c] row1[b]), (a, b, c) cyclic
#pragma unroll
      for (int a0 = 0; a0 < 3; a0++) {
        const int b0 = (a0 + 1) % 3, c0 = (a0 + 2) % 3;
        cpx<float> t = csub(cmul(u[b0], u[3 + c0]), cmul(u[c0], u[3 + b0]));
        d[6 + a0] = {-0.5f * t.re, 0.5f * t.im};
      }
    }
  }
}

// neighbour scales of the FP16S/BF16S formats folded into the accumulating
// fma (1, default) or multiplied into the link product first (0)
#ifndef ODWF_SCALE_IN_FMA
#define ODWF_SCALE_IN_FMA 1
#endif

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

// the same with every term scaled by sc, the per-site scale of a neighbour
// stored with one: acc += sc [g; -SIG B^dag g], each real one fma
template <int MU, int SIG>
__device__ __forceinline__ void reconstruct_scaled(const cpx<float> (&g)[6], float sc, cpx<float> (&acc)[12]) {
  using B = GammaB<MU>;
  constexpr int q0 = B::p0, q1 = B::p1;
  constexpr int fq0 = (q0 == 0) ? B::f0 : B::f1;
  constexpr int fq1 = (q1 == 0) ? B::f0 : B::f1;
  const float sl = SIG > 0 ? -sc : sc;  // the lower components enter with -SIG
#pragma unroll
  for (int c = 0; c < 3; c++) {
    acc[c] = {fmaf(sc, g[c].re, acc[c].re), fmaf(sc, g[c].im, acc[c].im)};
    acc[3 + c] = {fmaf(sc, g[3 + c].re, acc[3 + c].re), fmaf(sc, g[3 + c].im, acc[3 + c].im)};
    const cpx<float> l0 = mulf<ConjCode<fq0>::v>(g[q0 * 3 + c]);
    const cpx<float> l1 = mulf<ConjCode<fq1>::v>(g[q1 * 3 + c]);
    acc[6 + c] = {fmaf(sl, l0.re, acc[6 + c].re), fmaf(sl, l0.im, acc[6 + c].im)};
    acc[9 + c] = {fmaf(sl, l1.re, acc[9 + c].re), fmaf(sl, l1.im, acc[9 + c].im)};
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

// the same hop for a neighbour stored with a per-site scale: the projection and
// the link product are linear, so the scale enters only where the terms are
// accumulated (one fma per real instead of a product and a sum)
template <int MU, int SIG, class R>
__device__ __forceinline__ void hop_one_scaled(const cpx<R> (&psi)[12], R sc, const cpx<R>* U,
                                               cpx<R> (&acc)[12]) {
  cpx<R> h[6], g[6];
  project<MU, SIG>(psi, h);
  su3_mul(U, h, g);
  if constexpr (ODWF_SCALE_IN_FMA && sizeof(R) == 4) {
    reconstruct_scaled<MU, SIG>(g, sc, acc);
  } else {
#pragma unroll
    for (int k = 0; k < 6; k++) g[k] = cscale(sc, g[k]);
    reconstruct<MU, SIG>(g, acc);
  }
}

// first site of this block under the configured traversal
//
// Tiled walk (tile_y, tile_z > 0): a tile is tile_x x-row segments (of spb
// half-row sites) by tile_y by tile_z rows, walked segment-fastest, then y, z,
// with t innermost over tile_t slices (all of t when 0), so that the t
// neighbours a slice reads were fetched by the slices just before it.
// xcd = 1: hardware dispatches block b to XCD b % 8; XCD x is given the
// contiguous logical range [start(x), start(x) + count(x)), one run of tiles
// per XCD.  xcd = 2 (lockstep): the eight XCDs walk the eight tiles of a
// group of xgy (y) x 8 / xgy (z) adjacent tiles at the same time, block for
// block, so the halo rows two XCDs share are fetched by both at about the same
// time and the second read is served by the memory-side cache.
__device__ __forceinline__ long block_first_site(const HopArgs& a) {
  int lb = blockIdx.x;
  const int hx = a.L[0] >> 1;
  if (a.tile_y > 0) {
    const int nseg = hx / a.spb;
    const int tx = a.tile_x > 0 ? a.tile_x : nseg;
    const int tlen = a.tile_t > 0 ? a.tile_t : a.L[3];
    const int nty = a.L[1] / a.tile_y, ntz = a.L[2] / a.tile_z, ntx = nseg / tx;
    int rest, tyi, tzi;
    if (a.xcd == 2) {
      const int per = tx * a.tile_y * a.tile_z * tlen;  // blocks of one tile
      const int x = lb & 7, k = lb >> 3;
      const int xgy = a.xcd_gy, xgz = 8 / a.xcd_gy;
      const int gy = x % xgy, gz = x / xgy;  // this XCD's tile in the group
      int r2 = k % per;
      int grp = k / per;
      const int seg_i = r2 % tx;
      r2 /= tx;
      const int yi = r2 % a.tile_y;
      r2 /= a.tile_y;
      const int zi = r2 % a.tile_z;
      const int tl = r2 / a.tile_z;
      // groups: xgy x xgz tiles in (y, z), then x tiles, then t chunks
      const int ngy = nty / xgy, ngz = ntz / xgz;
      tyi = (grp % ngy) * xgy + gy;
      grp /= ngy;
      tzi = (grp % ngz) * xgz + gz;
      grp /= ngz;
      const int txi = grp % ntx;
      const int tc = grp / ntx;
      const int y = tyi * a.tile_y + yi, z = tzi * a.tile_z + zi, t = tc * tlen + tl;
      const int seg = txi * tx + seg_i;
      return (((long)t * a.L[2] + z) * a.L[1] + y) * hx + (long)seg * a.spb;
    }
    if (a.xcd) {
      const int q = a.nblocks >> 3, rem = a.nblocks & 7;
      const int x = lb & 7, k = lb >> 3;
      lb = x * q + min(x, rem) + k;
    }
    rest = lb;
    const int seg_i = rest % tx;
    rest /= tx;
    const int yi = rest % a.tile_y;
    rest /= a.tile_y;
    const int zi = rest % a.tile_z;
    rest /= a.tile_z;
    const int tl = rest % tlen;
    rest /= tlen;
    tyi = rest % nty;
    rest /= nty;
    tzi = rest % ntz;
    rest /= ntz;
    const int txi = rest % ntx;
    rest /= ntx;
    const int y = tyi * a.tile_y + yi, z = tzi * a.tile_z + zi;
    const int t = rest * tlen + tl;  // rest: index of the t chunk
    const int seg = txi * tx + seg_i;
    return (((long)t * a.L[2] + z) * a.L[1] + y) * hx + (long)seg * a.spb;
  }
  if (a.xcd) {
    const int q = a.nblocks >> 3, rem = a.nblocks & 7;
    const int x = lb & 7, k = lb >> 3;
    lb = x * q + min(x, rem) + k;
  }
  return (long)lb * a.spb;
}

#ifndef ODWF_HOP_GROUP64
#define ODWF_HOP_GROUP64 2
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

// the fused epilogue's own-site streams (x term, CG residual, output) are read
// or written once per launch: nontemporal (1, default), so that they do not
// displace the neighbour rows the hop re-reads from L2; 0: plain accesses
#ifndef ODWF_NT_FUSED
#define ODWF_NT_FUSED 1
#endif

// x term of the fused epilogue: already transformed in the column buffer, or
// loaded here (and transformed here when it has a fifth-dimension program)
enum XMode { X_LDS = 1, X_LOAD = 2 };

// Fused epilogue of one output site after the hop: the fifth-dimension column
// passes, the x term, the norm for the partial sums, and the residual, the CG
// update or the store.  Every thread of the block calls it (the column passes
// synchronise the block); returns this lane's share of the partial sum.
template <class P, int NS>
__device__ __forceinline__ double fused_tail(const HopArgs& a, cpx<typename P::real> (&acc)[12], bool valid,
                                             long j, int sl, int r, int s, int nsb,
                                             cpx<typename P::real>* buf, const typename P::real* coef,
                                             const typename P::real* kap, int xmode) {
  using R = typename P::real;
  constexpr int NSP = NS + 1;
  const int nrhs = a.nrhs;
  auto column_pass = [&](const M5Prog& prog, cpx<R>(&v)[12]) {
    if constexpr (LanePass<R, NS>::on) {
      // the column lives in the lanes of this (site, rhs): no LDS, no barrier
      m5_run_lanes<NS>(prog, v, coef, kap[r], s);
      return;
    }
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

  if (a.prog_h.n > 0) column_pass(a.prog_h, acc);  // never together with X_LDS
  const int cgmode = a.partial ? (a.cg_r ? 2 : (a.cg_p ? 3 : 1)) : 0;
  const bool cg_update = cgmode == 2 && valid && a.scal[r].active;
  cpx<R> xv[12], rv[12];
  bool r_loaded = false;
  const bool has_x = a.xin != nullptr;
  if (has_x) {
    if (xmode == X_LDS) {  // transformed before the hop, still in the column buffer
      if (valid) {
        const cpx<R>* b = buf + ((size_t)(sl * nrhs + r) * 12) * NSP + s;
#pragma unroll
        for (int c = 0; c < 12; c++) xv[c] = b[c * NSP];
      }
    } else {
      if (valid) load_site<P, ODWF_NT_FUSED>(a.xin, a.xin_sc, j, r, s, nrhs, NS, xv);
      if constexpr (LanePass<R, NS>::on && !P::SCALED) {
        // the CG residual travels with the x term: one memory round trip fewer
        if (cg_update) {
          load_site<P, ODWF_NT_FUSED>(a.cg_r, a.cg_r_sc, j, r, s, nrhs, NS, rv);
          r_loaded = true;
        }
      }
      if (a.prog_x.n > 0) column_pass(a.prog_x, xv);
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
    if (cg_update) {
      const R al = (R)a.scal[r].alpha;
      {  // r -= alpha N p, |r|^2
        if (!r_loaded) load_site<P, ODWF_NT_FUSED>(a.cg_r, a.cg_r_sc, j, r, s, nrhs, NS, rv);
#pragma unroll
        for (int c = 0; c < 12; c++) {
          rv[c] = csub(rv[c], cscale(al, acc[c]));
          nval += (double)cnorm2(rv[c]);
        }
        store_site<P, ODWF_NT_FUSED>(a.cg_r, a.cg_r_sc, j, r, s, nrhs, NS, rv);
      }
      // x += alpha p runs in the vector step after beta (vec_cg_step_kernel),
      // which reads p there anyway
    }
  } else if (valid && a.out) {
    store_site<P, ODWF_NT_FUSED>(a.out, a.out_sc, j, r, s, nrhs, NS, acc);
  }

  return nval;
}

// FP16 storage: the spin projection reads the stored halves directly.  Each
// real of h = psi_up -/+ f psi_dn (f in {+-1, +-i}) is one fma(+-1, dn, up) of
// the two halves (v_fma_mix_f32 converts and adds in one instruction); it
// rounds exactly as the sum of the converted values.  `one` is 1.0 held where
// the compiler cannot fold it (a product by the literal 1.0 would turn back
// into a conversion and an add).
template <int CODE, int SIG>
__device__ __forceinline__ cpx<float> proj_h16(uint32_t up, uint32_t dn, float one) {
  const __half2 u = *reinterpret_cast<const __half2*>(&up), d = *reinterpret_cast<const __half2*>(&dn);
  const float ur = __low2float(u), ui = __high2float(u), dr = __low2float(d), di = __high2float(d);
  const float m = SIG > 0 ? -one : one;  // h = up + m (f dn)
  if constexpr (CODE == 0) return {fmaf(m, dr, ur), fmaf(m, di, ui)};
  if constexpr (CODE == 1) return {fmaf(-m, dr, ur), fmaf(-m, di, ui)};
  if constexpr (CODE == 2) return {fmaf(-m, di, ur), fmaf(m, dr, ui)};
  return {fmaf(m, di, ur), fmaf(-m, dr, ui)};
}
template <int MU, int SIG>
__device__ __forceinline__ void hop_one_h16(const uint32_t (&w)[12], float sc, float one, const cpx<float>* U,
                                            cpx<float> (&acc)[12]) {
  using B = GammaB<MU>;
  cpx<float> h[6], g[6];
#pragma unroll
  for (int c = 0; c < 3; c++) {
    h[c] = proj_h16<B::f0, SIG>(w[c], w[(2 + B::p0) * 3 + c], one);
    h[3 + c] = proj_h16<B::f1, SIG>(w[3 + c], w[(2 + B::p1) * 3 + c], one);
  }
  su3_mul(U, h, g);
  if constexpr (ODWF_SCALE_IN_FMA) {
    reconstruct_scaled<MU, SIG>(g, sc, acc);
  } else {
#pragma unroll
    for (int k = 0; k < 6; k++) g[k] = cscale(sc, g[k]);
    reconstruct<MU, SIG>(g, acc);
  }
}
template <bool DAG>
__device__ __forceinline__ void hop_dir_h16(int dir, const uint32_t (&w)[12], float sc, float one,
                                            const cpx<float>* U, cpx<float> (&acc)[12]) {
  const bool minus = (dir < 4) != DAG;
  const cpx<float>* Ud = U + dir * 9;
  switch (dir & 3) {
    case 0: if (minus) hop_one_h16<0, +1>(w, sc, one, Ud, acc); else hop_one_h16<0, -1>(w, sc, one, Ud, acc); break;
    case 1: if (minus) hop_one_h16<1, +1>(w, sc, one, Ud, acc); else hop_one_h16<1, -1>(w, sc, one, Ud, acc); break;
    case 2: if (minus) hop_one_h16<2, +1>(w, sc, one, Ud, acc); else hop_one_h16<2, -1>(w, sc, one, Ud, acc); break;
    default: if (minus) hop_one_h16<3, +1>(w, sc, one, Ud, acc); else hop_one_h16<3, -1>(w, sc, one, Ud, acc); break;
  }
}

// one neighbour's hopping term: acc += (1 -/+ gamma_mu) U psi for the
// direction dir (0-3 forward, 4-7 backward); the scaled formats carry the
// neighbour's per-site scale sc separately
template <class P, bool DAG>
__device__ __forceinline__ void hop_dir(int dir, const cpx<typename P::real> (&psi)[12], typename P::real sc,
                                        const cpx<typename P::real>* U, cpx<typename P::real> (&acc)[12]) {
  // forward hop: (1 - gamma) for W, (1 + gamma) for W^dag; backward swapped
  const bool minus = (dir < 4) != DAG;
  const cpx<typename P::real>* Ud = U + dir * 9;
  if constexpr (P::SCALED) {
    switch (dir & 3) {
      case 0: if (minus) hop_one_scaled<0, +1>(psi, sc, Ud, acc); else hop_one_scaled<0, -1>(psi, sc, Ud, acc); break;
      case 1: if (minus) hop_one_scaled<1, +1>(psi, sc, Ud, acc); else hop_one_scaled<1, -1>(psi, sc, Ud, acc); break;
      case 2: if (minus) hop_one_scaled<2, +1>(psi, sc, Ud, acc); else hop_one_scaled<2, -1>(psi, sc, Ud, acc); break;
      default: if (minus) hop_one_scaled<3, +1>(psi, sc, Ud, acc); else hop_one_scaled<3, -1>(psi, sc, Ud, acc); break;
    }
  } else {
    switch (dir & 3) {
      case 0: if (minus) hop_one<0, +1>(psi, Ud, acc); else hop_one<0, -1>(psi, Ud, acc); break;
      case 1: if (minus) hop_one<1, +1>(psi, Ud, acc); else hop_one<1, -1>(psi, Ud, acc); break;
      case 2: if (minus) hop_one<2, +1>(psi, Ud, acc); else hop_one<2, -1>(psi, Ud, acc); break;
      default: if (minus) hop_one<3, +1>(psi, Ud, acc); else hop_one<3, -1>(psi, Ud, acc); break;
    }
  }
}

// a block-uniform integer in a scalar register (the compiler does not always
// prove uniformity through the traversal arithmetic)
__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

// The eight hopping terms of output site j0 + sl of a block that lies inside
// one x-row (half-row length a multiple of the sites per block), summed into
// acc (the factor -1/2 rides on the staged links).  y, z, t and the parity of
// the row are then block-uniform: the seven neighbour rows (own row for the x
// hops, y +- 1, z +- 1, t +- 1) are scalar 64-bit bases, and a lane addresses a
// neighbour as base + one of three 32-bit offsets (own column, x + 1, x - 1)
// + a constant chunk offset, so the loads need almost no vector address
// arithmetic.  Terms are summed in the order +x, -x, +y, -y, +z, -z, +t, -t,
// the neighbours loaded G at a time ahead of their arithmetic.
template <class P, int NS, bool DAG>
__device__ __forceinline__ void hop_sum_row(const HopArgs& a, int j0, int sl, int r, int s,
                                            const cpx<typename P::real>* U, cpx<typename P::real> (&acc)[12]) {
  using R = typename P::real;
  constexpr int NCG = 12 / P::CPB;
  const int nrhs = a.nrhs;
  const int L1 = a.L[1], L2 = a.L[2], L3 = a.L[3];
  const int hx = a.L[0] >> 1;
  const int jb = uniform_int(j0);
  const int xh0 = jb % hx;
  const int row = jb / hx;
  const int y = row % L1;
  const int z = (row / L1) % L2;
  const int t = row / (L1 * L2);
  const int p = (y + z + t + a.out_par) & 1;
  const int yp = y + 1 == L1 ? 0 : y + 1, ym = y == 0 ? L1 - 1 : y - 1;
  const int zp = z + 1 == L2 ? 0 : z + 1, zm = z == 0 ? L2 - 1 : z - 1;
  const int tp = t + 1 == L3 ? 0 : t + 1, tm = t == 0 ? L3 - 1 : t - 1;
  // per lane: half-row column of the own site and of its x neighbours
  // (x + 1 lies in column xi (p = 0) or xi + 1 (p = 1); x - 1 in xi - 1 or xi)
  const int xi = xh0 + sl;
  const int xip = p ? (xi + 1 == hx ? 0 : xi + 1) : xi;
  const int xim = p ? xi : (xi == 0 ? hx - 1 : xi - 1);
  auto boff = [&](int q) { return (unsigned)((((q * nrhs + r) * NCG) * NS + s) * 16); };
  const unsigned off_own = boff(xi), off_xp = boff(xip), off_xm = boff(xim);
  const size_t row_bytes = (size_t)hx * nrhs * NCG * NS * 16;
  auto soff = [&](int q) { return (unsigned)(((q * nrhs + r) * NS + s) * 4); };
  const unsigned soff_own = soff(xi), soff_xp = soff(xip), soff_xm = soff(xim);
  const size_t srow_bytes = (size_t)hx * nrhs * NS * 4;
  const bool flip_f = a.bc_t < 0 && t + 1 == L3;  // forward t hop wraps
  const bool flip_b = a.bc_t < 0 && t == 0;       // backward t hop wraps
  const unsigned char* in = reinterpret_cast<const unsigned char*>(a.in);
  const unsigned char* in_sc = reinterpret_cast<const unsigned char*>(a.in_sc);
  // FP16 neighbours stay packed until the projection (see proj_h16)
  constexpr bool RAW16 = std::is_same<P, SP16>::value;
  using Nb = typename std::conditional<RAW16, uint32_t[12], cpx<R>[12]>::type;
  float one = 1.0f;
  if constexpr (RAW16) asm("s_mov_b32 %0, 1.0" : "=s"(one));
  // neighbour of direction dir (0-3 forward, 4-7 backward) into v; sc its scale
  auto load_nb = [&](int dir, Nb& v, R& sc) {
    const int mu = dir & 3;
    const bool fwd = dir < 4;
    const int yy = mu == 1 ? (fwd ? yp : ym) : y;
    const int zz = mu == 2 ? (fwd ? zp : zm) : z;
    const int tt = mu == 3 ? (fwd ? tp : tm) : t;
    const int nrow = (tt * L2 + zz) * L1 + yy;  // block-uniform
    const unsigned off = mu == 0 ? (fwd ? off_xp : off_xm) : off_own;
    const unsigned char* base = in + (size_t)nrow * row_bytes;
    uint4 q[NCG];
#pragma unroll
    for (int cg = 0; cg < NCG; cg++) q[cg] = *reinterpret_cast<const uint4*>(base + off + cg * NS * 16);
    if constexpr (RAW16) {
#pragma unroll
      for (int cg = 0; cg < NCG; cg++) {
        v[cg * 4 + 0] = q[cg].x;
        v[cg * 4 + 1] = q[cg].y;
        v[cg * 4 + 2] = q[cg].z;
        v[cg * 4 + 3] = q[cg].w;
      }
    } else {
#pragma unroll
      for (int cg = 0; cg < NCG; cg++) unpack_chunk<P>(q[cg], &v[cg * P::CPB]);
    }
    if constexpr (P::SCALED) {
      const unsigned so = mu == 0 ? (fwd ? soff_xp : soff_xm) : soff_own;
      sc = *reinterpret_cast<const float*>(in_sc + (size_t)nrow * srow_bytes + so);
    } else {
      sc = R(1);
    }
  };
  // its hopping term, with the boundary sign of a wrapping t hop
  auto apply_nb = [&](int dir, Nb& v, R sc) {
    if ((dir == 3 && flip_f) || (dir == 7 && flip_b)) {
      if constexpr (P::SCALED) {
        sc = -sc;
      } else {
#pragma unroll
        for (int c = 0; c < 12; c++) v[c] = {-v[c].re, -v[c].im};
      }
    }
    if constexpr (RAW16) hop_dir_h16<DAG>(dir, v, sc, one, U, acc);
    else hop_dir<P, DAG>(dir, v, sc, U, acc);
  };
  constexpr int G = HopGroup<P>::G;
  // direction of the k-th term: 0, 4, 1, 5, 2, 6, 3, 7
  auto dir_of = [](int k) { return (k >> 1) | ((k & 1) << 2); };
  // (a rolled loop: unrolled, the compiler issues the loads of later groups
  // early and spills them at the register budget of four waves per SIMD; a
  // software pipeline over two register buffers fits three waves and was
  // slower in the fused kernels)
#pragma unroll 1
  for (int g0 = 0; g0 < 8; g0 += G) {
    Nb psi[G];
    R scl[G];
#pragma unroll
    for (int k = 0; k < G; k++) load_nb(dir_of(g0 + k), psi[k], scl[k]);
#pragma unroll
    for (int k = 0; k < G; k++) apply_nb(dir_of(g0 + k), psi[k], scl[k]);
  }
}

// The eight hopping terms of output site j, summed into acc (the factor -1/2
// rides on the staged links), for any block shape: the coordinates and the
// neighbour index are formed per lane.
template <class P, int NS, bool DAG>
__device__ __forceinline__ void hop_sum(const HopArgs& a, long j, int r, int s,
                                        const cpx<typename P::real>* U, cpx<typename P::real> (&acc)[12]) {
  using R = typename P::real;
  const int nrhs = a.nrhs;
  const int L0 = a.L[0], L1 = a.L[1], L2 = a.L[2], L3 = a.L[3];
  const int hx = L0 >> 1;
  const int xh = (int)(j % hx);
  long rest = j / hx;
  const int y = (int)(rest % L1);
  rest /= L1;
  const int z = (int)(rest % L2);
  const int t = (int)(rest / L2);
  const int x = 2 * xh + ((y + z + t + a.out_par) & 1);
  const bool flip_f = a.bc_t < 0 && t + 1 == L3;  // forward t hop wraps
  const bool flip_b = a.bc_t < 0 && t == 0;       // backward t hop wraps
  constexpr int G = HopGroup<P>::G;
  // direction order: +x, -x, +y, -y, ... (4-7 are the backward hops)
#pragma unroll 1
  for (int g0 = 0; g0 < 8; g0 += G) {
    cpx<R> psi[G][12];
    R scl[G];  // per-site scales of the neighbours (scaled formats)
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
      if constexpr (P::SCALED) load_site_cached_raw<P>(a.in, a.in_sc, nj, r, s, nrhs, NS, psi[k], scl[k]);
      else {
        load_site_cached<P>(a.in, a.in_sc, nj, r, s, nrhs, NS, psi[k]);
        scl[k] = R(1);
      }
    }
#pragma unroll
    for (int k = 0; k < G; k++) {
      const int dir = ((g0 + k) >> 1) | (((g0 + k) & 1) << 2);
      if ((dir == 3 && flip_f) || (dir == 7 && flip_b)) {
        if constexpr (P::SCALED) {
          scl[k] = -scl[k];
        } else {
#pragma unroll
          for (int c = 0; c < 12; c++) psi[k][c] = {-psi[k][c].re, -psi[k][c].im};
        }
      }
      hop_dir<P, DAG>(dir, psi[k], scl[k], U, acc);
    }
  }
}

// fifth-dimension coefficients of the lane-parallel programs staged in LDS
// (1, default) or read from global memory (0)
#ifndef ODWF_LDS_COEF
#define ODWF_LDS_COEF 1
#endif
// minimum waves per SIMD the register allocation must allow (the fused FP32
// kernels fit four when their column programs run across lanes)
#ifndef ODWF_HOP_WAVES32
#define ODWF_HOP_WAVES32 4
#endif
#ifndef ODWF_HOP_WAVES64
#define ODWF_HOP_WAVES64 2
#endif
template <class P, int NS, bool PLAIN>
struct HopWaves {
  static constexpr int W = sizeof(typename P::real) == 8
                               ? ODWF_HOP_WAVES64
                               : ((PLAIN || LanePass<typename P::real, NS>::on) ? ODWF_HOP_WAVES32 : 2);
};

template <class P, int NS, bool DAG, bool PLAIN>
__global__ void __launch_bounds__(256, (HopWaves<P, NS, PLAIN>::W)) hop_kernel(const HopArgs a) {
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
  const R* coef = reinterpret_cast<const R*>(a.coef);
  if (!PLAIN && tid < nrhs) kap[tid] = (R)a.kappa[tid];
  // the lane-parallel programs read their coefficients at every step: from a
  // copy in the (otherwise unused) column buffer those are LDS reads
  R* coef_lds = reinterpret_cast<R*>(buf);
  if constexpr (!PLAIN && LanePass<R, NS>::on && ODWF_LDS_COEF)
    for (int i = tid; i < 2 * NCOEF * NS; i += blockDim.x) coef_lds[i] = coef[i];
  stage_links<P>(a.links, j0, nsb, lnk);

  cpx<R> xv[12];
  const bool has_x = !PLAIN && a.xin != nullptr;
  // x term with its own fifth-dimension program: transform it in LDS before the
  // hop, so no column pass runs while the hop accumulators are live
  // (with the lane-parallel programs the x term is transformed after the hop instead)
  const bool x_first = has_x && a.prog_x.n > 0 && !LanePass<R, NS>::on;
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
    const cpx<R>* U = lnk + (size_t)sl * 8 * 9;
    // (row offsets are 32-bit: a row of a half field is at most 3 MB here)
    if ((a.L[0] >> 1) % a.spb == 0 && a.L[0] <= 256) hop_sum_row<P, NS, DAG>(a, (int)j0, sl, r, s, U, acc);
    else hop_sum<P, NS, DAG>(a, j, r, s, U, acc);
  }
  if constexpr (PLAIN) {
    if (valid) store_site<P, ODWF_NT_STORE>(a.out, a.out_sc, j, r, s, nrhs, NS, acc);
    return;
  }

  // the own-site index again from the block-uniform first site: cheaper than
  // keeping the 64-bit index live through the hop (which spills at 4 waves);
  // the empty asm stops the compiler from reusing the value computed earlier
  int slr = sl;
  asm volatile("" : "+v"(slr));
  const double nval = fused_tail<P, NS>(a, acc, valid, j0 + slr, sl, r, s, nsb, buf,
                                        (LanePass<R, NS>::on && ODWF_LDS_COEF) ? coef_lds : coef, kap,
                                        x_first ? X_LDS : X_LOAD);
  if (a.partial) block_reduce_rhs(valid ? nval : 0.0, NS, a.spb, nrhs, red, a.partial, blockIdx.x);
}


// threads per block of the plain hop: FP64 rows are twice as long, and 8-site
// segments (128 threads at Ns = 16) fetch 20 % less and run 5 % faster at
// 64^4 x 16; in FP32 they fetch 10 % less in the same time
#ifndef ODWF_HOP_THREADS64
#define ODWF_HOP_THREADS64 128
#endif
#ifndef ODWF_HOP_THREADS32
#define ODWF_HOP_THREADS32 256
#endif

// extra LDS per block (plain / fused kernels): caps the blocks resident per CU
#ifndef ODWF_HOP_SMEM_PAD
#define ODWF_HOP_SMEM_PAD 0
#endif
#ifndef ODWF_HOP_SMEM_PAD_F
#define ODWF_HOP_SMEM_PAD_F 0
#endif
template <class P, int NS>
static size_t hop_smem(int spb, int nrhs, int block, bool plain) {
  using R = typename P::real;
  const size_t lnk_n = (size_t)spb * 8 * 9;
  const size_t buf_n = plain ? 0 : (size_t)spb * nrhs * 12 * (NS + 1);
  const size_t region = (lnk_n + buf_n) * sizeof(cpx<R>);
  size_t off = (region + MAXRHS * sizeof(R) + 15) & ~size_t(15);
  return off + (size_t)(block + 16 * MAXRHS) * sizeof(double) +
         (plain ? ODWF_HOP_SMEM_PAD : ODWF_HOP_SMEM_PAD_F);
}

template <class P, int NS>
static hipError_t launch_hop_t(HopArgs a, int dag, hipStream_t st) {
  const int inner = a.nrhs * NS;
  if (inner > 256 || a.nrhs > MAXRHS) return hipErrorInvalidValue;
  const bool plain = a.prog_h.n == 0 && a.prog_o.n == 0 && a.xin == nullptr && a.partial == nullptr &&
                     a.c_h == 1.0;
  // plain launches (no partial sums) may use smaller blocks: shorter x-row
  // segments, so more of them per XCD share its L2
  const int threads = !plain ? 256 : (sizeof(typename P::real) == 8 ? ODWF_HOP_THREADS64 : ODWF_HOP_THREADS32);
  a.spb = threads >= inner ? threads / inner : 1;
  const int block = (a.spb * inner + 63) & ~63;  // whole waves, <= 256
  a.nblocks = (int)((a.h + a.spb - 1) / a.spb);
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
