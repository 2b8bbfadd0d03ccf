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

// the same hop for a neighbour stored with a per-site scale: the projection and
// the link product are linear, so the scale multiplies the 6 numbers of g
// instead of the 12 of the spinor
template <int MU, int SIG, class R>
__device__ __forceinline__ void hop_one_scaled(const cpx<R> (&psi)[12], R sc, const cpx<R>* U,
                                               cpx<R> (&acc)[12]) {
  cpx<R> h[6], g[6];
  project<MU, SIG>(psi, h);
  su3_mul(U, h, g);
#pragma unroll
  for (int k = 0; k < 6; k++) g[k] = cscale(sc, g[k]);
  reconstruct<MU, SIG>(g, acc);
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
      if (valid) load_site<P>(a.xin, a.xin_sc, j, r, s, nrhs, NS, xv);
      if constexpr (LanePass<R, NS>::on && !P::SCALED) {
        // the CG residual travels with the x term: one memory round trip fewer
        if (cg_update) {
          load_site<P>(a.cg_r, a.cg_r_sc, j, r, s, nrhs, NS, rv);
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
        if (!r_loaded) load_site<P>(a.cg_r, a.cg_r_sc, j, r, s, nrhs, NS, rv);
#pragma unroll
        for (int c = 0; c < 12; c++) {
          rv[c] = csub(rv[c], cscale(al, acc[c]));
          nval += (double)cnorm2(rv[c]);
        }
        store_site<P>(a.cg_r, a.cg_r_sc, j, r, s, nrhs, NS, rv);
      }
      // x += alpha p runs in the vector step after beta (vec_cg_step_kernel),
      // which reads p there anyway
    }
  } else if (valid && a.out) {
    store_site<P, ODWF_NT_STORE>(a.out, a.out_sc, j, r, s, nrhs, NS, acc);
  }

  return nval;
}

// The eight hopping terms of output site j, summed into acc (times -1/2).
// ROW: the block lies inside one x-row (half-row length a multiple of the
// sites per block), so y, z, t and the parity of the row are block-uniform;
// every neighbour is then read as a block-uniform row base (64-bit, scalar
// registers) plus a per-lane 32-bit byte offset, and only three such offsets
// exist per lane: the own column (y, z, t hops) and the two x neighbours.
// Otherwise the coordinates and the neighbour index are formed per lane.
template <class P, int NS, bool DAG, bool ROW>
__device__ __forceinline__ void hop_sum(const HopArgs& a, long j0, long j, int sl, int r, int s,
                                        const cpx<typename P::real>* U, cpx<typename P::real> (&acc)[12]) {
  using R = typename P::real;
  constexpr int NCG = 12 / P::CPB;
  const int nrhs = a.nrhs;
  const int L0 = a.L[0], L1 = a.L[1], L2 = a.L[2], L3 = a.L[3];
  const int hx = L0 >> 1;
  int x, y, z, t;
  // ROW only: per-lane byte offsets within a row of the chunk and scale arrays
  unsigned off_own = 0, off_xp = 0, off_xm = 0, soff_own = 0, soff_xp = 0, soff_xm = 0;
  size_t row_bytes = 0, srow_bytes = 0;
  if constexpr (ROW) {
    const int xh0 = (int)j0 % hx;
    const int row = (int)j0 / hx;
    y = row % L1;
    z = (row / L1) % L2;
    t = row / (L1 * L2);
    const int p = (y + z + t + a.out_par) & 1;
    const int xi = xh0 + sl;
    x = 2 * xi + p;
    // x + 1 lies in half-row column xi (p = 0) or xi + 1 (p = 1); x - 1 in xi - 1 or xi
    const int xip = p ? (xi + 1 == hx ? 0 : xi + 1) : xi;
    const int xim = p ? xi : (xi == 0 ? hx - 1 : xi - 1);
    auto boff = [&](int q) { return (unsigned)((((q * nrhs + r) * NCG) * NS + s) * 16); };
    auto soff = [&](int q) { return (unsigned)(((q * nrhs + r) * NS + s) * 4); };
    off_own = boff(xi);
    off_xp = boff(xip);
    off_xm = boff(xim);
    row_bytes = (size_t)hx * nrhs * NCG * NS * 16;
    if constexpr (P::SCALED) {
      soff_own = soff(xi);
      soff_xp = soff(xip);
      soff_xm = soff(xim);
      srow_bytes = (size_t)hx * nrhs * NS * 4;
    }
  } else {
    const int xh = (int)(j % hx);
    long rest = j / hx;
    y = (int)(rest % L1);
    rest /= L1;
    z = (int)(rest % L2);
    t = (int)(rest / L2);
    x = 2 * xh + ((y + z + t + a.out_par) & 1);
  }
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
      if constexpr (ROW) {
        int yy = y, zz = z, tt = t;
        if (mu == 1) yy = fwd ? (y + 1 == L1 ? 0 : y + 1) : (y == 0 ? L1 - 1 : y - 1);
        if (mu == 2) zz = fwd ? (z + 1 == L2 ? 0 : z + 1) : (z == 0 ? L2 - 1 : z - 1);
        if (mu == 3) tt = fwd ? (t + 1 == L3 ? 0 : t + 1) : (t == 0 ? L3 - 1 : t - 1);
        const int nrow = (tt * L2 + zz) * L1 + yy;
        const unsigned off = mu == 0 ? (fwd ? off_xp : off_xm) : off_own;
        const unsigned char* base = reinterpret_cast<const unsigned char*>(a.in) + (size_t)nrow * row_bytes;
        uint4 q[NCG];
#pragma unroll
        for (int cg = 0; cg < NCG; cg++)
          q[cg] = *reinterpret_cast<const uint4*>(base + off + (size_t)cg * NS * 16);
#pragma unroll
        for (int cg = 0; cg < NCG; cg++) unpack_chunk<P>(q[cg], &psi[k][cg * P::CPB]);
        if constexpr (P::SCALED) {
          const unsigned so = mu == 0 ? (fwd ? soff_xp : soff_xm) : soff_own;
          scl[k] = *reinterpret_cast<const float*>(reinterpret_cast<const unsigned char*>(a.in_sc) +
                                                   (size_t)nrow * srow_bytes + so);
        } else {
          scl[k] = R(1);
        }
      } else {
        int xx = x, yy = y, zz = z, tt = t;
        if (mu == 0) xx = fwd ? (x + 1 == L0 ? 0 : x + 1) : (x == 0 ? L0 - 1 : x - 1);
        if (mu == 1) yy = fwd ? (y + 1 == L1 ? 0 : y + 1) : (y == 0 ? L1 - 1 : y - 1);
        if (mu == 2) zz = fwd ? (z + 1 == L2 ? 0 : z + 1) : (z == 0 ? L2 - 1 : z - 1);
        if (mu == 3) tt = fwd ? (t + 1 == L3 ? 0 : t + 1) : (t == 0 ? L3 - 1 : t - 1);
        const long nj = (((long)tt * L2 + zz) * L1 + yy) * hx + (xx >> 1);
        if constexpr (P::SCALED) load_site_cached_raw<P>(a.in, a.in_sc, nj, r, s, nrhs, NS, psi[k], scl[k]);
        else load_site_cached<P>(a.in, a.in_sc, nj, r, s, nrhs, NS, psi[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < G; k++) {
      const int dir = ((g0 + k) >> 1) | (((g0 + k) & 1) << 2);
      const bool fwd = dir < 4;
      if ((dir == 3 && flip_f) || (dir == 7 && flip_b)) {
        if constexpr (P::SCALED) {
          scl[k] = -scl[k];
        } else {
#pragma unroll
          for (int c = 0; c < 12; c++) psi[k][c] = {-psi[k][c].re, -psi[k][c].im};
        }
      }
      // forward hop: (1 - gamma) for W, (1 + gamma) for W^dag; backward swapped
      const bool minus = fwd != DAG;
      if constexpr (P::SCALED) {
        const R sc = scl[k];
        switch (dir & 3) {
          case 0: if (minus) hop_one_scaled<0, +1>(psi[k], sc, U + dir * 9, acc); else hop_one_scaled<0, -1>(psi[k], sc, U + dir * 9, acc); break;
          case 1: if (minus) hop_one_scaled<1, +1>(psi[k], sc, U + dir * 9, acc); else hop_one_scaled<1, -1>(psi[k], sc, U + dir * 9, acc); break;
          case 2: if (minus) hop_one_scaled<2, +1>(psi[k], sc, U + dir * 9, acc); else hop_one_scaled<2, -1>(psi[k], sc, U + dir * 9, acc); break;
          default: if (minus) hop_one_scaled<3, +1>(psi[k], sc, U + dir * 9, acc); else hop_one_scaled<3, -1>(psi[k], sc, U + dir * 9, acc); break;
        }
      } else {
        switch (dir & 3) {
          case 0: if (minus) hop_one<0, +1>(psi[k], U + dir * 9, acc); else hop_one<0, -1>(psi[k], U + dir * 9, acc); break;
          case 1: if (minus) hop_one<1, +1>(psi[k], U + dir * 9, acc); else hop_one<1, -1>(psi[k], U + dir * 9, acc); break;
          case 2: if (minus) hop_one<2, +1>(psi[k], U + dir * 9, acc); else hop_one<2, -1>(psi[k], U + dir * 9, acc); break;
          default: if (minus) hop_one<3, +1>(psi[k], U + dir * 9, acc); else hop_one<3, -1>(psi[k], U + dir * 9, acc); break;
        }
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 12; c++) acc[c] = cscale(R(-0.5), acc[c]);
}

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
    if ((a.L[0] >> 1) % a.spb == 0 && a.L[0] <= 256) hop_sum<P, NS, DAG, true>(a, j0, j, sl, r, s, U, acc);
    else hop_sum<P, NS, DAG, false>(a, j0, j, sl, r, s, U, acc);
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
  const double nval = fused_tail<P, NS>(a, acc, valid, j0 + slr, sl, r, s, nsb, buf, coef, kap,
                                        x_first ? X_LDS : X_LOAD);
  if (a.partial) block_reduce_rhs(valid ? nval : 0.0, NS, a.spb, nrhs, red, a.partial, blockIdx.x);
}


// ---------------------------------------------------------------------------
// t-sweep hopping kernel.  Block b owns the output sites of one x-row segment
// (seg, y, z) for t in [t0, t0 + sweep) and walks them in t.  The input
// spinor of the block's own column at t is carried from step to step in
// registers: it is the x-hop input at step t (one of the two x neighbours of
// every output site lies in the own column, the other in the adjacent lane,
// exchanged through LDS), the +t neighbour at step t - 1 and, as its projected
// half spinor, the -t neighbour at step t + 1.  Each input row of the column is
// therefore read from memory once per sweep instead of three times; the y and
// z neighbours are the own columns of concurrently running blocks and are
// read while they are still in L2.  The epilogue of every step is the one of
// the one-t-per-block kernel.
// ---------------------------------------------------------------------------
#ifndef ODWF_SWEEP_WAVES_PLAIN
#define ODWF_SWEEP_WAVES_PLAIN 2
#endif
// minimum waves per SIMD of the t-sweep kernel (its column state costs registers)
template <class P, bool PLAIN>
struct SweepWaves {
  static constexpr int W = sizeof(typename P::real) == 8 ? (PLAIN ? 2 : 1) : (PLAIN ? ODWF_SWEEP_WAVES_PLAIN : 2);
};

template <class P, int NS, bool DAG, bool PLAIN>
__global__ void __launch_bounds__(256, (SweepWaves<P, PLAIN>::W)) hop_sweep_kernel(const HopArgs a) {
  using R = typename P::real;
  extern __shared__ __align__(16) unsigned char smem[];
  const int nrhs = a.nrhs;
  const int inner = nrhs * NS;
  const int tid = threadIdx.x;
  const int sl = tid / inner;
  const int lr = tid - sl * inner;
  const int r = lr / NS;
  const int s = lr - r * NS;
  if (!gate_any(a.gate, a.gate_mode, nrhs)) {
    // idle block: its partial-sum slots still have to read zero
    if (a.partial && tid < nrhs) {
      a.partial[(long)blockIdx.x * nrhs + tid] = 0.0;
      for (int k = 1; k < a.sweep; k++)
        a.partial[((long)gridDim.x + (long)blockIdx.x * (a.sweep - 1) + (k - 1)) * nrhs + tid] = 0.0;
    }
    return;
  }
  const int L0 = a.L[0], L1 = a.L[1], L2 = a.L[2], L3 = a.L[3];
  const int hx = L0 >> 1;
  const int spb = a.spb;
  const int nseg = hx / spb;

  // block -> (segment, y, z, first t): XCD-aware ranges, (y, z) tiles, t chunks slowest
  int lb = blockIdx.x;
  if (a.xcd) {
    const int q = a.nblocks >> 3, rem = a.nblocks & 7;
    const int xc = lb & 7, k = lb >> 3;
    lb = xc * q + min(xc, rem) + k;
  }
  const int ty = a.tile_y > 0 ? a.tile_y : 1, tz = a.tile_z > 0 ? a.tile_z : 1;
  const int seg = lb % nseg;
  lb /= nseg;
  const int yi = lb % ty;
  lb /= ty;
  const int zi = lb % tz;
  lb /= tz;
  const int nty = L1 / ty, ntz = L2 / tz;
  const int y = (lb % nty) * ty + yi;
  lb /= nty;
  const int z = (lb % ntz) * tz + zi;
  lb /= ntz;
  const int t0 = lb * a.sweep;

  // padded threads have sl >= spb; gated-off right-hand sides do no work
  const bool valid = sl < spb && gate_on(a.gate, a.gate_mode, r);
  const int xh = seg * spb + sl;  // half-row index of this lane's output and own input column
  constexpr int NSP = NS + 1;

  // LDS: links, the x-exchange buffer (spb + 2 sites: the segment and one
  // halo site on each side) aliased with the column buffer, kappa, reduction scratch
  const size_t lnk_n = (size_t)spb * 8 * 9;
  const int xstride = (spb + 2) * inner;  // per component
  const size_t xch_n = (size_t)12 * xstride;
  const size_t col_n = (size_t)spb * nrhs * 12 * NSP;
  const size_t buf_n = PLAIN || xch_n > col_n ? xch_n : col_n;
  cpx<R>* lnk = reinterpret_cast<cpx<R>*>(smem);
  cpx<R>* buf = lnk + lnk_n;
  const size_t region = (lnk_n + buf_n) * sizeof(cpx<R>);
  R* kap = reinterpret_cast<R*>(smem + region);
  double* red = reinterpret_cast<double*>(smem + ((region + MAXRHS * sizeof(R) + 15) & ~size_t(15)));
  const R* coef = reinterpret_cast<const R*>(a.coef);
  if (!PLAIN && tid < nrhs) kap[tid] = (R)a.kappa[tid];

  auto row = [&](int tt, int zz, int yy) { return (((long)tt * L2 + zz) * L1 + yy) * hx; };
  // sign of the +t and -t hops: forward (1 - gamma_t) for W, (1 + gamma_t) for W^dag
  constexpr int SIG_TF = DAG ? -1 : +1;
  constexpr int SIG_TB = DAG ? +1 : -1;
  const int yp = y + 1 == L1 ? 0 : y + 1, ym = y == 0 ? L1 - 1 : y - 1;
  const int zp = z + 1 == L2 ? 0 : z + 1, zm = z == 0 ? L2 - 1 : z - 1;
  const int xslot = (sl + 1) * inner + lr;  // this lane's column in the exchange buffer

  // column state: cur = input at (xh, t); hm = projected -t term for the output at t
  cpx<R> cur[12];
  cpx<R> hm[6];
  if (valid) {
    load_site_row<P>(a.in, a.in_sc, row(t0, z, y), xh, r, s, nrhs, NS, cur);
    cpx<R> pv[12];
    load_site_row<P>(a.in, a.in_sc, row(t0 == 0 ? L3 - 1 : t0 - 1, z, y), xh, r, s, nrhs, NS, pv);
    if (t0 == 0 && a.bc_t < 0) {
#pragma unroll
      for (int c = 0; c < 12; c++) pv[c] = {-pv[c].re, -pv[c].im};
    }
    project<3, SIG_TB>(pv, hm);
  }
  double nval = 0.0;

#pragma unroll 1
  for (int t = t0; t < t0 + a.sweep; t++) {
    const long rt = row(t, z, y);
    const long j0 = rt + (long)seg * spb;
    const long j = j0 + sl;
    // the output site sits at x = 2 xh + shift: the own column is its +x
    // neighbour when shift = 0 (the -x one is the previous lane's column), and
    // its -x neighbour when shift = 1 (the +x one is the next lane's column)
    const int shift = (y + z + t + a.out_par) & 1;
    __syncthreads();  // readers of the previous step's links and buffers are done
    stage_links<P>(a.links, j0, spb, lnk);
    if (sl < spb) {
#pragma unroll
      for (int c = 0; c < 12; c++) buf[(size_t)c * xstride + xslot] = cur[c];
      // halo: the column beyond the segment edge on the side this step needs
      const bool edge = shift ? sl == spb - 1 : sl == 0;
      if (edge && gate_on(a.gate, a.gate_mode, r)) {
        const int xo = shift ? (xh + 1 == hx ? 0 : xh + 1) : (xh == 0 ? hx - 1 : xh - 1);
        cpx<R> o[12];
        load_site_row<P>(a.in, a.in_sc, rt, xo, r, s, nrhs, NS, o);
        const int hs = xslot + (shift ? inner : -inner);
#pragma unroll
        for (int c = 0; c < 12; c++) buf[(size_t)c * xstride + hs] = o[c];
      }
    }
    __syncthreads();

    cpx<R> acc[12];
#pragma unroll
    for (int c = 0; c < 12; c++) acc[c] = {R(0), R(0)};
    cpx<R> nxt[12];
    if (valid) {
      const cpx<R>* U = lnk + (size_t)sl * 8 * 9;
      // terms summed in the order +x, -x, +y, -y, +z, -z, +t, -t, as in the
      // one-t-per-block kernel, so that both round alike
      {
        cpx<R> o[12];
        const int sp = xslot + (shift ? inner : 0), sm = xslot - (shift ? 0 : inner);
#pragma unroll
        for (int c = 0; c < 12; c++) o[c] = buf[(size_t)c * xstride + sp];
        hop_one<0, DAG ? -1 : +1>(o, U + 0 * 9, acc);
#pragma unroll
        for (int c = 0; c < 12; c++) o[c] = buf[(size_t)c * xstride + sm];
        hop_one<0, DAG ? +1 : -1>(o, U + 4 * 9, acc);
      }
      // y and z hops from the neighbouring columns, one direction pair per round
#pragma unroll 1
      for (int mu = 1; mu <= 2; mu++) {
        cpx<R> pp[12], pm[12];
        load_site_row<P>(a.in, a.in_sc, mu == 1 ? row(t, z, yp) : row(t, zp, y), xh, r, s, nrhs, NS, pp);
        load_site_row<P>(a.in, a.in_sc, mu == 1 ? row(t, z, ym) : row(t, zm, y), xh, r, s, nrhs, NS, pm);
        if (mu == 1) {
          hop_one<1, DAG ? -1 : +1>(pp, U + 1 * 9, acc);
          hop_one<1, DAG ? +1 : -1>(pm, U + 5 * 9, acc);
        } else {
          hop_one<2, DAG ? -1 : +1>(pp, U + 2 * 9, acc);
          hop_one<2, DAG ? +1 : -1>(pm, U + 6 * 9, acc);
        }
      }
      {  // +t: the next input of the own column
        load_site_row<P>(a.in, a.in_sc, row(t + 1 == L3 ? 0 : t + 1, z, y), xh, r, s, nrhs, NS, nxt);
        if (t + 1 == L3 && a.bc_t < 0) {
#pragma unroll
          for (int c = 0; c < 12; c++) nxt[c] = {-nxt[c].re, -nxt[c].im};
        }
        hop_one<3, SIG_TF>(nxt, U + 3 * 9, acc);
      }
      {  // -t: the projected input of the previous step
        cpx<R> g[6];
        su3_mul(U + 7 * 9, hm, g);
        reconstruct<3, SIG_TB>(g, acc);
      }
#pragma unroll
      for (int c = 0; c < 12; c++) acc[c] = cscale(R(-0.5), acc[c]);
      // the -t term of the next output is this step's own input
      cpx<R> o[12];
#pragma unroll
      for (int c = 0; c < 12; c++) o[c] = buf[(size_t)c * xstride + xslot];
      project<3, SIG_TB>(o, hm);
    }

    if constexpr (PLAIN) {
      if (valid) store_site<P>(a.out, a.out_sc, j, r, s, nrhs, NS, acc);
    } else {
      __syncthreads();  // the x-exchange buffer becomes the column buffer
      nval += fused_tail<P, NS>(a, acc, valid, j, sl, r, s, spb, buf, coef, kap, X_LOAD);
    }
    if (valid) {
#pragma unroll
      for (int c = 0; c < 12; c++) cur[c] = nxt[c];
    }
  }

  if (!PLAIN && a.partial) {
    // one slot for the whole sweep, zeros in the slots of the other steps so
    // that the partial array has the layout of the one-t-per-block kernel
    block_reduce_rhs(valid ? nval : 0.0, NS, spb, nrhs, red, a.partial, blockIdx.x);
    if (tid < nrhs) {
      for (int k = 1; k < a.sweep; k++)
        a.partial[((long)gridDim.x + (long)blockIdx.x * (a.sweep - 1) + (k - 1)) * nrhs + tid] = 0.0;
    }
  }
}

// extra LDS per block (plain / fused kernels): caps the blocks resident per CU
#ifndef ODWF_HOP_SMEM_PAD
#define ODWF_HOP_SMEM_PAD 0
#endif
#ifndef ODWF_HOP_SMEM_PAD_F
#define ODWF_HOP_SMEM_PAD_F 0
#endif
template <class P, int NS>
static size_t hop_smem(int spb, int nrhs, int block, bool plain, bool sweep) {
  using R = typename P::real;
  const size_t lnk_n = (size_t)spb * 8 * 9;
  const size_t col_n = plain ? 0 : (size_t)spb * nrhs * 12 * (NS + 1);
  const size_t xch_n = (size_t)12 * (spb + 2) * nrhs * NS;  // x-exchange buffer with halo
  const size_t buf_n = sweep ? (xch_n > col_n ? xch_n : col_n) : col_n;
  const size_t region = (lnk_n + buf_n) * sizeof(cpx<R>);
  size_t off = (region + MAXRHS * sizeof(R) + 15) & ~size_t(15);
  return off + (size_t)(block + 16 * MAXRHS) * sizeof(double) +
         (plain ? ODWF_HOP_SMEM_PAD : ODWF_HOP_SMEM_PAD_F);
}

template <class P, int NS>
static hipError_t launch_hop_t(HopArgs a, int dag, hipStream_t st) {
  const int inner = a.nrhs * NS;
  if (inner > 256 || a.nrhs > MAXRHS) return hipErrorInvalidValue;
  a.spb = 256 / inner;
  const int block = (a.spb * inner + 63) & ~63;  // whole waves, <= 256
  const bool plain = a.prog_h.n == 0 && a.prog_o.n == 0 && a.xin == nullptr && a.partial == nullptr &&
                     a.c_h == 1.0;
  const int hx = a.L[0] / 2;
  const bool sweep = a.sweep > 0 && hx % a.spb == 0 && a.L[3] % a.sweep == 0 &&
                     (a.tile_y <= 0 || a.L[1] % a.tile_y == 0) && (a.tile_z <= 0 || a.L[2] % a.tile_z == 0);
  if (sweep) {
    a.nblocks = (int)(a.h / a.spb / a.sweep);
    const size_t sm = hop_smem<P, NS>(a.spb, a.nrhs, block, plain, true);
    if (plain) {
      if (dag) hipLaunchKernelGGL((hop_sweep_kernel<P, NS, true, true>), dim3(a.nblocks), dim3(block), sm, st, a);
      else hipLaunchKernelGGL((hop_sweep_kernel<P, NS, false, true>), dim3(a.nblocks), dim3(block), sm, st, a);
    } else {
      if (dag) hipLaunchKernelGGL((hop_sweep_kernel<P, NS, true, false>), dim3(a.nblocks), dim3(block), sm, st, a);
      else hipLaunchKernelGGL((hop_sweep_kernel<P, NS, false, false>), dim3(a.nblocks), dim3(block), sm, st, a);
    }
    return hipGetLastError();
  }
  a.sweep = 0;
  a.nblocks = (int)((a.h + a.spb - 1) / a.spb);
  const size_t sm = hop_smem<P, NS>(a.spb, a.nrhs, block, plain, false);
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
