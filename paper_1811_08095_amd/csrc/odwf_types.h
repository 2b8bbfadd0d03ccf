// Plain data types shared by the host runtime and the HIP kernels of libodwf.
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace odwf {

constexpr int MAXRHS = 16;  // right-hand sides per multi-RHS launch
// reliable-update trigger of the FP32 inner CG: recompute the true residual in
// FP64 once the iterated |r| falls below delta * max |r| since the last update;
// delta = 0.01 (measured at 64^3 x 64 x 16: the same iteration count as 0.1
// with half the updates; 0.001 starts to add iterations)
constexpr double RELIABLE_DELTA2 = 1e-4;
// right-hand sides per launch for a given Ns (Ns * nrhs lanes per site <= 256)
inline int max_rhs_per_launch(int Ns) { return 256 / Ns < MAXRHS ? 256 / Ns : MAXRHS; }

enum Prec { PREC64 = 0, PREC32 = 1, PREC16 = 2, PRECB16 = 3 };

// ---- fifth-dimension programs ---------------------------------------------
// Each operator acting on the fifth dimension is a product of diagonal scalings
// and cyclic bidiagonal matrices (or their inverses) with corner factor kappa =
// -mu, applied per chirality in the chirality-local index order.
enum M5Type : int8_t {
  M5_NOP = 0,
  M5_SCALE = 1,     // y_s *= d_s
  M5_MUL_LO = 2,    // y_s = d_s y_s + e_s y_{s-1},  y_0 = d_0 y_0 + kappa e_0 y_{N-1}
  M5_SOLVE_LO = 3,  // inverse of MUL_LO; d holds the reciprocal diagonal
  M5_MUL_UP = 4,    // y_s = d_s y_s + e_s y_{s+1},  y_{N-1} = d y + kappa e_{N-1} y_0
  M5_SOLVE_UP = 5   // inverse of MUL_UP; d holds the reciprocal diagonal
};

// coefficient arrays, each of length Ns, per chirality (chirality - mirrored)
enum CoefId : int8_t {
  CF_ONE = 0,       // 1
  CF_MONE = 1,      // -1
  CF_OMEGA = 2,     // omega_s
  CF_OMEGA_INV = 3, // 1 / omega_s
  CF_A = 4,         // a_s = (4 - m0) omega_s + 1
  CF_A_INV = 5,     // 1 / a_s
  CF_C = 6,         // c_s = (4 - m0) omega_s - 1
  CF_CSHIFT = 7,    // c_{s+1} (s < N-1), c_0 at s = N-1
  NCOEF = 8
};

struct M5Op {
  int8_t type, d, e, pad;
};
struct M5Prog {
  int n;
  M5Op op[4];
};

// ---- CG scalars, one record per right-hand side ----------------------------
struct CGScal {
  double rr;      // |r|^2 of the iterated residual
  double pAp;     // <p, N p> = |S p|^2
  double alpha;   // step length of the current iteration (0 when inactive)
  double beta;    // search-direction factor (0 when inactive)
  double f2;      // |f|^2 of the right-hand side of the iterated system
  double tol2;    // tol^2
  double rmax2;   // max |r|^2 since the last reliable update (mixed solves)
  double delta2;  // reliable-update threshold factor squared (0: never)
  int active;     // 1 while iterating
  int converged;  // iterated residual reached tol
  int nan;        // NaN/Inf met
  int update;     // reliable update requested
  int iters;      // iterations done
  int maxiter;    // iteration cap
  int confirm;    // 1: iterated convergence or maxiter requests a true-residual update
  int nupd;       // true-residual (reliable) updates this right-hand side iterated into
  int upd_iters;  // iteration count at its last true-residual update
};

// which right-hand sides a gated kernel works on
enum GateMode { GATE_NONE = 0, GATE_ACTIVE = 1, GATE_UPDATE = 2 };

struct KappaArr {
  double v[MAXRHS];  // per right-hand side: -mu_r
};

// ---- arguments of the fused hopping kernel ----------------------------------
struct HopArgs {
  const void* in;       // opposite-parity input half
  const float* in_sc;
  const void* links;    // links of the output parity
  void* out;            // output half
  float* out_sc;
  const void* xin;      // same-parity input for the x term
  const float* xin_sc;
  // fused CG residual update (CG mode 2): r -= alpha out, |r|^2; cg_p is the
  // right-hand side f of a residual f - out (CG mode 3)
  void* cg_r;
  float* cg_r_sc;
  const void* cg_p;
  const float* cg_p_sc;
  const CGScal* scal;
  double* partial;      // per block, per right-hand side
  const void* coef;     // [2][NCOEF][Ns], compute precision
  double kappa[MAXRHS]; // per right-hand side: -mu_r
  M5Prog prog_h;        // applied to the hopping result
  M5Prog prog_x;        // applied to the x term
  M5Prog prog_o;        // applied to the combination
  double c_h, c_x;      // combination c_h * prog_h(W in) + c_x * prog_x(x)
  int h, nrhs, spb, out_par, bc_t, dag;
  int L[4];
  int nblocks;
  // block traversal: xcd != 0 gives each of the 8 XCDs a contiguous range of
  // logical blocks, xcd = 2 walks groups of 8 adjacent (y, z) tiles with one
  // tile per XCD in lockstep; tile_y, tile_z > 0 walk (x-row segments,
  // y, z) tiles with t innermost so that t-neighbours are re-read while still
  // in L2; tile_x > 0 is the number of x-row segments of a tile (all of the
  // row when 0); tile_t > 0 cuts t into chunks of that length, each chunk
  // walking all tiles before the next chunk starts
  int xcd, tile_y, tile_z, tile_t, tile_x;
  int xcd_gy;  // xcd = 2: tiles of a lockstep group along y (1, 2, 4 or 8)
  // gating: lanes of right-hand sides not selected by gate_mode do no work
  const CGScal* gate;
  int gate_mode;
};

}  // namespace odwf
