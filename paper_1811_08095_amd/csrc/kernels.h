// Host-side launchers of the libodwf HIP kernels.  All launches are
// asynchronous on the given stream; they return the launch status.
#pragma once
#include <hip/hip_runtime.h>

#include "odwf_types.h"

namespace odwf {

struct Geom {
  int L[4];  // Lx, Ly, Lz, Lt
  long V, h;
};

// hopping kernel (hop.hip)
hipError_t launch_hop(const HopArgs& a, int prec, int Ns, hipStream_t st);
int hop_nblocks(int h, int nrhs, int Ns);

// layouts (pack.hip)
// canonical complex128 [rhs][s][t][z][y][x][4][3] (rhs offset r0, nrhs of them)
// <-> internal half of parity `par`.
hipError_t launch_pack_spinor(int prec, const void* canon, int r0, void* out, float* out_sc,
                              int par, int nrhs, int Ns, const Geom& g, hipStream_t st);
hipError_t launch_unpack_spinor(int prec, const void* in, const float* in_sc, void* canon, int r0,
                                int par, int nrhs, int Ns, const Geom& g, hipStream_t st);
// zero the sites of parity par of a canonical field (rhs r0 .. r0+nrhs-1)
hipError_t launch_zero_canon_parity(void* canon, int r0, int par, int nrhs, int Ns, const Geom& g,
                                    hipStream_t st);
// boundary maps of the effective 4D operator on canonical complex128 fields:
// embed 4D q [r][site][12] into 5D f [r][s][site][12] (chirality minus into
// slice 0, plus into slice Ns - 1, zeros elsewhere); project back
hipError_t launch_boundary_embed(const void* q, void* f, int nrhs, int Ns, const Geom& g, hipStream_t st);
hipError_t launch_boundary_project(const void* f, void* q, int nrhs, int Ns, const Geom& g, hipStream_t st);
// gauge: canonical complex128 [t][z][y][x][mu][3][3] -> per-parity link
// arrays [h][8][18 doubles] (prec64) or [h][8][12 floats] (reduced)
hipError_t launch_pack_gauge(const void* canon, void* out, int par, int prec, const Geom& g,
                             hipStream_t st);

// fifth-dimension programs on a half field (m5.hip), FP64 or FP32 storage:
// out = c0 * prog(in) + c1 * other   (other may be null)
hipError_t launch_m5(int prec, const void* in, const float* in_sc, void* out, float* out_sc,
                     const void* other, const float* other_sc, double c0, double c1,
                     const M5Prog& prog, const void* coef, const KappaArr& kappa, long h, int nrhs,
                     int Ns, hipStream_t st);

// BLAS-1 on half fields (blas.hip); n5 = h * nrhs * Ns five-dimensional sites
// gate / gate_mode (GateMode) restrict the work to selected right-hand sides
hipError_t launch_vec_zero(int prec, void* v, float* sc, long h, int nrhs, int Ns, hipStream_t st,
                           const CGScal* gate = nullptr, int gate_mode = GATE_NONE);
// dst = src (accumulate: dst += src), converting storage precision
hipError_t launch_vec_convert(int prec_src, const void* src, const float* src_sc, int prec_dst,
                              void* dst, float* dst_sc, int accumulate, long h, int nrhs, int Ns,
                              hipStream_t st, const CGScal* gate = nullptr, int gate_mode = GATE_NONE);
// one right-hand side of a field into one right-hand side of another (zeros if src null)
hipError_t launch_vec_copy_rhs(int prec_src, const void* src, const float* src_sc, int nrhs_src,
                               int r_src, int prec_dst, void* dst, float* dst_sc, int nrhs_dst,
                               int r_dst, long h, int Ns, hipStream_t st);
// CG vector step: x += alpha_r p for right-hand sides that iterated (alpha != 0),
// then p = r + beta_r p for the active ones
hipError_t launch_vec_cg_step(int prec, const void* r, const float* r_sc, void* p, float* p_sc, void* x,
                              float* x_sc, const CGScal* scal, long h, int nrhs, int Ns, hipStream_t st);
// per-block partial sums of |v|^2 per right-hand side
hipError_t launch_vec_norm2(int prec, const void* v, const float* sc, double* partial, long h,
                            int nrhs, int Ns, int* nblocks_out, hipStream_t st);
int vec_nblocks(long h, int nrhs, int Ns);

// fermion force of Re <chi, W psi> on the links of the sites of parity `par`
// (force.hip): own / nb are FP64 one-right-hand-side halves of chi and psi on
// parity par and on the other parity; F canonical [t][z][y][x][mu][3][3]
hipError_t launch_force(const void* chi_own, const void* psi_own, const void* chi_nb, const void* psi_nb,
                        const void* links, void* F, int par, int Ns, int bc_t, int accumulate, const Geom& g,
                        hipStream_t st);

// scalar finalisation (blas.hip), one block
enum FinKind { FIN_SUM = 0, FIN_ALPHA = 1, FIN_BETA = 2, FIN_INIT = 3, FIN_F2 = 4, FIN_TRUE = 5 };
// bytes a partial-sum buffer for nblocks blocks needs (includes the second
// reduction stage used for long partial arrays)
size_t partial_bytes(int nblocks, int nrhs);
// gated != 0: only right-hand sides whose update flag is set are finalised
hipError_t launch_fin(int kind, const double* partial, int nblocks, int nrhs, CGScal* scal,
                      double* out, hipStream_t st, int gated = 0);

}  // namespace odwf
