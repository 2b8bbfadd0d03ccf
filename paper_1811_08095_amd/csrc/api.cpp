// C ABI of libodwf: lattices, solvers, operator application and the
// even-odd preconditioned CG solves (FP64, FP32 with FP64 reliable updates,
// FP16/BF16 storage with FP64 defect correction).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "runtime.h"
#include "solver.h"

using namespace odwf;

namespace odwf {
hipError_t noalloc_init(int device);
void* noalloc_scratch(int device);
const char* last_error_cstr();
void prof_enable(int on);
void prof_read(long long* launches, double* ms, double* bytes);
void prof_read_kernel(int prec, int dag, long long* launches, double* ms, double* bytes);
}  // namespace odwf

#define HIPCHK(expr)                                                               \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) {                                                        \
      set_error(std::string("HIP error in ") + #expr + ": " + hipGetErrorString(e_)); \
      return ODWF_EHIP;                                                            \
    }                                                                              \
  } while (0)

#define REQUIRE(cond, msg)       \
  do {                           \
    if (!(cond)) {               \
      set_error(msg);            \
      return ODWF_EINVAL;        \
    }                            \
  } while (0)

static bool ns_supported(int Ns) { return Ns == 4 || Ns == 8 || Ns == 16 || Ns == 32; }

// ------------------------------------------------------------------------------
// lattices
// ------------------------------------------------------------------------------

extern "C" odwf_status odwf_lattice_create(const int dims[4], int bc_t, int device,
                                           odwf_lattice* out) {
  REQUIRE(dims && out, "odwf_lattice_create: null argument");
  for (int d = 0; d < 4; d++)
    REQUIRE(dims[d] >= 2 && dims[d] % 2 == 0 && dims[d] <= 4096,
            "odwf_lattice_create: every extent must be even, >= 2 and <= 4096");
  REQUIRE(bc_t == 1 || bc_t == -1, "odwf_lattice_create: bc_t must be +1 or -1");
  const long V = (long)dims[0] * dims[1] * dims[2] * dims[3];
  REQUIRE(V / 2 <= (1L << 30), "odwf_lattice_create: lattice too large");
  int ndev = 0;
  HIPCHK(hipGetDeviceCount(&ndev));
  REQUIRE(device >= 0 && device < ndev, "odwf_lattice_create: bad device index");
  HIPCHK(hipSetDevice(device));
  // set-up of the device: the address of the allocation-free entry point's
  // scratch array on this device (once per device)
  HIPCHK(noalloc_init(device));
  odwf_lattice L = new odwf_lattice_s();
  for (int d = 0; d < 4; d++) {
    L->dims[d] = dims[d];
    L->g.L[d] = dims[d];
  }
  L->bc_t = bc_t;
  L->device = device;
  L->g.V = V;
  L->g.h = V / 2;
  *out = L;
  return ODWF_OK;
}

extern "C" odwf_status odwf_lattice_load_gauge(odwf_lattice L, const void* U, int on_device,
                                               void* stream) {
  REQUIRE(L && U, "odwf_lattice_load_gauge: null argument");
  HIPCHK(hipSetDevice(L->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const size_t canon_bytes = (size_t)L->g.V * 4 * 9 * 16;
  const void* src = U;
  void* tmp = nullptr;
  if (!on_device) {
    if (hipMalloc(&tmp, canon_bytes) != hipSuccess) {
      (void)hipGetLastError();
      set_error("odwf_lattice_load_gauge: out of device memory for staging");
      return ODWF_ENOMEM;
    }
    HIPCHK(hipMemcpyAsync(tmp, U, canon_bytes, hipMemcpyHostToDevice, st));
    src = tmp;
  }
  const size_t b64 = (size_t)L->g.h * 8 * 18 * sizeof(double);
  const size_t b32 = (size_t)L->g.h * 8 * 12 * sizeof(float);
  for (int p = 0; p < 2; p++) {
    if (!L->U64[p] && hipMalloc(&L->U64[p], b64) != hipSuccess) {
      (void)hipGetLastError();
      L->U64[p] = nullptr;
      if (tmp) (void)hipFree(tmp);
      set_error("odwf_lattice_load_gauge: out of device memory");
      return ODWF_ENOMEM;
    }
    if (!L->U32[p] && hipMalloc(&L->U32[p], b32) != hipSuccess) {
      (void)hipGetLastError();
      L->U32[p] = nullptr;
      if (tmp) (void)hipFree(tmp);
      set_error("odwf_lattice_load_gauge: out of device memory");
      return ODWF_ENOMEM;
    }
    HIPCHK(launch_pack_gauge(src, L->U64[p], p, PREC64, L->g, st));
    HIPCHK(launch_pack_gauge(src, L->U32[p], p, PREC32, L->g, st));
  }
  if (tmp) {
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipFree(tmp));
  }
  L->loaded = true;
  return ODWF_OK;
}

extern "C" odwf_status odwf_lattice_bytes(odwf_lattice L, size_t* bytes) {
  REQUIRE(L && bytes, "odwf_lattice_bytes: null argument");
  *bytes = (L->U64[0] ? 2 * (size_t)L->g.h * 8 * 18 * sizeof(double) : 0) +
           (L->U32[0] ? 2 * (size_t)L->g.h * 8 * 12 * sizeof(float) : 0);
  return ODWF_OK;
}

extern "C" void odwf_lattice_destroy(odwf_lattice L) {
  if (!L) return;
  (void)hipSetDevice(L->device);
  for (int p = 0; p < 2; p++) {
    if (L->U64[p]) (void)hipFree(L->U64[p]);
    if (L->U32[p]) (void)hipFree(L->U32[p]);
  }
  delete L;
}

// ------------------------------------------------------------------------------
// solvers
// ------------------------------------------------------------------------------

extern "C" odwf_status odwf_solver_create(odwf_lattice L, int Ns, double m0, const double* omega,
                                          odwf_solver* out) {
  REQUIRE(L && omega && out, "odwf_solver_create: null argument");
  REQUIRE(ns_supported(Ns), "odwf_solver_create: Ns must be 4, 8, 16 or 32");
  REQUIRE(std::isfinite(m0), "odwf_solver_create: m0 must be finite");
  for (int s = 0; s < Ns; s++)
    REQUIRE(std::isfinite(omega[s]) && omega[s] > 0, "odwf_solver_create: omega_s must be > 0");
  HIPCHK(hipSetDevice(L->device));
  odwf_solver S = new odwf_solver_s();
  S->lat = L;
  S->Ns = Ns;
  S->m0 = m0;
  S->omega.assign(omega, omega + Ns);
  // coefficient table [chi][id][q], chirality - in mirrored order
  std::vector<double> c64(2 * NCOEF * Ns);
  std::vector<float> c32(2 * NCOEF * Ns);
  const double k4 = 4.0 - m0;
  for (int chi = 0; chi < 2; chi++) {
    auto w = [&](int q) { return omega[chi ? Ns - 1 - q : q]; };
    for (int q = 0; q < Ns; q++) {
      const double a = k4 * w(q) + 1.0, c = k4 * w(q) - 1.0;
      const double cn = k4 * w(q + 1 < Ns ? q + 1 : 0) - 1.0;
      double v[NCOEF];
      v[CF_ONE] = 1.0;
      v[CF_MONE] = -1.0;
      v[CF_OMEGA] = w(q);
      v[CF_OMEGA_INV] = 1.0 / w(q);
      v[CF_A] = a;
      v[CF_A_INV] = 1.0 / a;
      v[CF_C] = c;
      v[CF_CSHIFT] = cn;
      for (int id = 0; id < NCOEF; id++) {
        c64[(chi * NCOEF + id) * Ns + q] = v[id];
        c32[(chi * NCOEF + id) * Ns + q] = (float)v[id];
      }
    }
  }
  if (hipMalloc(&S->coef64, c64.size() * sizeof(double)) != hipSuccess ||
      hipMalloc(&S->coef32, c32.size() * sizeof(float)) != hipSuccess) {
    (void)hipGetLastError();
    delete S;
    set_error("odwf_solver_create: out of device memory");
    return ODWF_ENOMEM;
  }
  HIPCHK(hipMemcpy(S->coef64, c64.data(), c64.size() * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(S->coef32, c32.data(), c32.size() * sizeof(float), hipMemcpyHostToDevice));
  *out = S;
  return ODWF_OK;
}

extern "C" void odwf_solver_destroy(odwf_solver S) {
  if (!S) return;
  (void)hipSetDevice(S->lat->device);
  (void)hipDeviceSynchronize();
  for (auto& kv : S->ws) delete kv.second;
  if (S->coef64) (void)hipFree(S->coef64);
  if (S->coef32) (void)hipFree(S->coef32);
  delete S;
}

// ------------------------------------------------------------------------------
// operator application
// ------------------------------------------------------------------------------

// the half fields each operator uses, as bits: input even (1), input odd (2),
// output even (4), output odd (8), even scratch (16), odd scratch (32)
static int apply_needs(odwf_op op) {
  const bool full = op == ODWF_OP_D || op == ODWF_OP_DDAG || op == ODWF_OP_DDAGD;
  int m = 0;
  if (op != ODWF_OP_HOP_EO) m |= 1;
  if (op != ODWF_OP_HOP_OE && op < ODWF_OP_SCHUR) m |= 2;
  if (op != ODWF_OP_HOP_OE) m |= 4;
  if (op == ODWF_OP_HOP_OE || op == ODWF_OP_M5INV || full) m |= 8;
  if (full || op == ODWF_OP_SCHUR_DAG || op == ODWF_OP_SCHUR_NORMAL) m |= 16;
  if (full || op >= ODWF_OP_SCHUR) m |= 32;
  return m;
}

// supplies the half field named `name` (nrhs right-hand sides, precision prec)
using HalfFn = std::function<HV(const char* name, int nrhs, int prec)>;

static odwf_status apply_chunk(odwf_solver S, odwf_op op, const double* mq, int prec, int r0,
                               int nrhs, const void* in, void* out, hipStream_t st,
                               const HalfFn& get, bool noprof) {
  const Geom& g = S->lat->g;
  const int Ns = S->Ns;
  OpCtx c;
  c.S = S;
  c.st = st;
  c.prec = prec;
  c.nrhs = nrhs;
  c.noprof = noprof;
  for (int r = 0; r < MAXRHS; r++) c.kappa[r] = r < nrhs ? -mq[r0 + r] / (2.0 * S->m0) : 0.0;
  const int needs = apply_needs(op);
  const bool need_ie = needs & 1, need_io = needs & 2, need_oe = needs & 4, need_oo = needs & 8;
  const bool need_te = needs & 16, need_to = needs & 32;
  auto half = [&](bool need, const char* name) { return need ? get(name, nrhs, prec) : HV(); };
  HV ie = half(need_ie, "ap.ie"), io = half(need_io, "ap.io");
  HV oe = half(need_oe, "ap.oe"), oo = half(need_oo, "ap.oo");
  HV te = half(need_te, "ap.te"), to = half(need_to, "ap.to");
  if ((need_ie && !ie.d) || (need_io && !io.d) || (need_oe && !oe.d) || (need_oo && !oo.d) ||
      (need_te && !te.d) || (need_to && !to.d)) {
    set_error("odwf_apply: out of device memory for workspaces");
    return ODWF_ENOMEM;
  }
  if (need_ie) HIPCHK(launch_pack_spinor(prec, in, r0, ie.d, ie.sc, 0, nrhs, Ns, g, st));
  if (need_io) HIPCHK(launch_pack_spinor(prec, in, r0, io.d, io.sc, 1, nrhs, Ns, g, st));
  bool have_e = true, have_o = true;
  HopOpt o;
  switch (op) {
    case ODWF_OP_HOP_EO:
      HIPCHK(hop(c, 0, 0, io, &oe, o));
      have_o = false;
      break;
    case ODWF_OP_HOP_OE:
      HIPCHK(hop(c, 1, 0, ie, &oo, o));
      have_e = false;
      break;
    case ODWF_OP_M5INV:
      HIPCHK(m5(c, ie, oe, prog_ainv()));
      HIPCHK(m5(c, io, oo, prog_ainv()));
      break;
    case ODWF_OP_D:
    case ODWF_OP_DDAGD:
      HIPCHK(apply_D(c, ie, io, te, to, oe, oo));
      if (op == ODWF_OP_DDAGD) {
        HIPCHK(apply_Ddag(c, oe, oo, te, to, ie, io));
        std::swap(oe, ie);
        std::swap(oo, io);
      }
      break;
    case ODWF_OP_DDAG:
      HIPCHK(apply_Ddag(c, ie, io, te, to, oe, oo));
      break;
    case ODWF_OP_SCHUR:
      HIPCHK(apply_schur(c, ie, to, oe));
      have_o = false;
      break;
    case ODWF_OP_SCHUR_DAG:
      HIPCHK(apply_schur_dag(c, ie, te, to, oe));
      have_o = false;
      break;
    case ODWF_OP_SCHUR_NORMAL:
      HIPCHK(apply_normal(c, ie, to, te, oe, nullptr));
      have_o = false;
      break;
    default:
      set_error("odwf_apply: unknown operator");
      return ODWF_EINVAL;
  }
  if (have_e) HIPCHK(launch_unpack_spinor(prec, oe.d, oe.sc, out, r0, 0, nrhs, Ns, g, st));
  else HIPCHK(launch_zero_canon_parity(out, r0, 0, nrhs, Ns, g, st));
  if (have_o) HIPCHK(launch_unpack_spinor(prec, oo.d, oo.sc, out, r0, 1, nrhs, Ns, g, st));
  else HIPCHK(launch_zero_canon_parity(out, r0, 1, nrhs, Ns, g, st));
  return ODWF_OK;
}

extern "C" odwf_status odwf_apply(odwf_solver S, odwf_op op, const double* mq, odwf_prec prec,
                                  int nrhs, const void* in, void* out, void* stream) {
  REQUIRE(S && mq && in && out, "odwf_apply: null argument");
  REQUIRE(nrhs >= 1, "odwf_apply: nrhs must be >= 1");
  REQUIRE(in != out, "odwf_apply: in and out must be distinct buffers");
  REQUIRE(prec >= ODWF_FP64 && prec <= ODWF_BF16S, "odwf_apply: bad precision");
  REQUIRE(S->lat->loaded, "odwf_apply: gauge field not loaded");
  for (int r = 0; r < nrhs; r++) REQUIRE(std::isfinite(mq[r]), "odwf_apply: mq must be finite");
  HIPCHK(hipSetDevice(S->lat->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lk(S->mtx);
  Workspace& W = S->workspace(st);
  const long h = S->lat->g.h;
  const int Ns = S->Ns;
  const HalfFn get = [&](const char* name, int n, int p) { return W.half(name, h, n, Ns, p); };
  const int chunk = max_rhs_per_launch(S->Ns);
  for (int r0 = 0; r0 < nrhs; r0 += chunk) {
    const int n = std::min(chunk, nrhs - r0);
    odwf_status s = apply_chunk(S, op, mq, (int)prec, r0, n, in, out, st, get, false);
    if (s != ODWF_OK) return s;
  }
  return ODWF_OK;
}

// bytes of one half field in the scratch array, rounded up to 256 bytes
static size_t scratch_half_bytes(long h, int nrhs, int Ns, int prec) {
  auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
  return up(half_bytes(h, nrhs, Ns, prec)) + up(scale_bytes(h, nrhs, Ns, prec));
}

extern "C" odwf_status odwf_apply_noalloc(odwf_solver S, odwf_op op, const double* mq,
                                          odwf_prec prec, int nrhs, const void* in, void* out,
                                          void* stream) {
  REQUIRE(S && mq && in && out, "odwf_apply_noalloc: null argument");
  REQUIRE(nrhs >= 1, "odwf_apply_noalloc: nrhs must be >= 1");
  REQUIRE(in != out, "odwf_apply_noalloc: in and out must be distinct buffers");
  REQUIRE(prec >= ODWF_FP64 && prec <= ODWF_BF16S, "odwf_apply_noalloc: bad precision");
  REQUIRE(op >= ODWF_OP_HOP_EO && op <= ODWF_OP_SCHUR_NORMAL, "odwf_apply_noalloc: unknown operator");
  REQUIRE(S->lat->loaded, "odwf_apply_noalloc: gauge field not loaded");
  for (int r = 0; r < nrhs; r++) REQUIRE(std::isfinite(mq[r]), "odwf_apply_noalloc: mq must be finite");
  const long h = S->lat->g.h;
  const int Ns = S->Ns;
  const int chunk = max_rhs_per_launch(Ns);
  const int n0 = std::min(chunk, nrhs);
  const int needs = apply_needs(op);
  int nhalves = 0;
  for (int b = 0; b < 6; b++) nhalves += (needs >> b) & 1;
  const size_t need = (size_t)nhalves * scratch_half_bytes(h, n0, Ns, (int)prec);
  if (need > ODWF_NOALLOC_SCRATCH_BYTES) {
    set_error("odwf_apply_noalloc: this operator needs " + std::to_string(need) +
              " bytes of scratch for " + std::to_string(n0) +
              " right-hand side(s) per launch; the maximum is " +
              std::to_string((size_t)ODWF_NOALLOC_SCRATCH_BYTES));
    return ODWF_ENOMEM;
  }
  HIPCHK(hipSetDevice(S->lat->device));
  unsigned char* base = static_cast<unsigned char*>(noalloc_scratch(S->lat->device));
  REQUIRE(base, "odwf_apply_noalloc: no scratch address for this device");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lk(S->mtx);
  size_t off = 0;
  // half fields carved one after another from the scratch array (every
  // element is written by a pack or an operator kernel before it is read, so
  // nothing has to start at zero)
  const HalfFn get = [&](const char*, int n, int p) {
    HV v;
    v.prec = p;
    v.d = base + off;
    const size_t db = (half_bytes(h, n, Ns, p) + 255) & ~size_t(255);
    const size_t sb = (scale_bytes(h, n, Ns, p) + 255) & ~size_t(255);
    v.sc = sb ? reinterpret_cast<float*>(base + off + db) : nullptr;
    off += db + sb;
    return v;
  };
  for (int r0 = 0; r0 < nrhs; r0 += chunk) {
    const int n = std::min(chunk, nrhs - r0);
    off = 0;
    odwf_status s = apply_chunk(S, op, mq, (int)prec, r0, n, in, out, st, get, true);
    if (s != ODWF_OK) return s;
  }
  return ODWF_OK;
}

// ------------------------------------------------------------------------------
// solves
// ------------------------------------------------------------------------------

extern "C" odwf_status odwf_solve(odwf_solver S, odwf_mode mode, const double* mq, const double* tol,
                                  int nrhs, odwf_prec inner, int maxiter, const void* b, void* x,
                                  int use_x0, odwf_stats* stats, void* stream) {
  REQUIRE(S && mq && tol && b && x, "odwf_solve: null argument");
  REQUIRE(nrhs >= 1, "odwf_solve: nrhs must be >= 1");
  REQUIRE(mode == ODWF_SOLVE_EO_NORMAL || mode == ODWF_SOLVE_FULL, "odwf_solve: bad mode");
  REQUIRE(inner >= ODWF_FP64 && inner <= ODWF_BF16S, "odwf_solve: bad inner precision");
  REQUIRE(maxiter >= 1, "odwf_solve: maxiter must be >= 1");
  REQUIRE(!(use_x0 && b == x), "odwf_solve: x may alias b only when use_x0 == 0");
  REQUIRE(S->lat->loaded, "odwf_solve: gauge field not loaded");
  for (int r = 0; r < nrhs; r++) {
    REQUIRE(std::isfinite(mq[r]), "odwf_solve: mq must be finite");
    REQUIRE(tol[r] > 0 && tol[r] < 1, "odwf_solve: tol must be in (0, 1)");
  }
  HIPCHK(hipSetDevice(S->lat->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lk(S->mtx);
  odwf_status worst = ODWF_OK;
  const int chunk = max_rhs_per_launch(S->Ns);
  for (int r0 = 0; r0 < nrhs; r0 += chunk) {
    const int n = std::min(chunk, nrhs - r0);
    odwf_status s = solve_chunk(S, (int)mode, mq + r0, tol + r0, r0, n, (int)inner, maxiter, b, x,
                                use_x0, stats ? stats + r0 : nullptr, st);
    if (s == ODWF_EHIP || s == ODWF_ENOMEM || s == ODWF_EINVAL) return s;
    if (s != ODWF_OK && worst == ODWF_OK) worst = s;
  }
  return worst;
}

// A single right-hand side's FP32 half field above this size does not stay in
// the memory-side cache (256 MB): multi-right-hand-side launches then lose
// more in neighbour re-fetch (their sites are nmass times larger) than they
// save in shared link reads, and the masses are solved one launch each
// (measured at 64^3 x 8 x 16 with six masses: shared launches 0.85x, at 32^4
// 0.91x, at 16^4 1.05x the speed of one mass at a time).
constexpr size_t MASSES_SHARED_MAX_HALF_BYTES = size_t(256) << 20;

extern "C" odwf_status odwf_solve_masses(odwf_solver S, const double* mq, const double* tol,
                                         int nmass, odwf_prec inner, int maxiter, const void* b,
                                         void* y, int use_y0, int per_launch, odwf_stats* stats,
                                         void* stream) {
  REQUIRE(S && mq && tol && b && y, "odwf_solve_masses: null argument");
  REQUIRE(nmass >= 1 && nmass <= max_rhs_per_launch(S->Ns),
          "odwf_solve_masses: nmass must be in [1, min(16, 256 / Ns)]");
  REQUIRE(per_launch >= 0 && per_launch <= nmass, "odwf_solve_masses: per_launch must be in [0, nmass]");
  REQUIRE(inner >= ODWF_FP64 && inner <= ODWF_BF16S, "odwf_solve_masses: bad inner precision");
  REQUIRE(maxiter >= 1, "odwf_solve_masses: maxiter must be >= 1");
  REQUIRE(b != y, "odwf_solve_masses: b and y must be distinct buffers");
  REQUIRE(S->lat->loaded, "odwf_solve_masses: gauge field not loaded");
  for (int k = 0; k < nmass; k++) {
    REQUIRE(std::isfinite(mq[k]), "odwf_solve_masses: mq must be finite");
    REQUIRE(tol[k] > 0 && tol[k] < 1, "odwf_solve_masses: tol must be in (0, 1)");
  }
  HIPCHK(hipSetDevice(S->lat->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lk(S->mtx);
  const long h = S->lat->g.h;
  const int Ns = S->Ns;
  if (per_launch == 0)
    per_launch = half_bytes(h, 1, Ns, PREC32) > MASSES_SHARED_MAX_HALF_BYTES ? 1 : nmass;
  SolveIO io;
  io.bcast_b = true;
  if (per_launch == nmass) {  // every mass in the same launches, straight into y
    io.y_packed = y;
    return solve_chunk(S, ODWF_SOLVE_EO_NORMAL, mq, tol, 0, nmass, (int)inner, maxiter, b, nullptr,
                       use_y0, stats, st, io);
  }
  // groups of per_launch masses, each solved in a packed field of its own and
  // copied into its slots of y
  Workspace& W = S->workspace(st);
  HV yg = W.half("m.y", h, per_launch, Ns, PREC64);
  if (!yg.d) {
    set_error("odwf_solve_masses: out of device memory for workspaces");
    return ODWF_ENOMEM;
  }
  io.y_packed = yg.d;
  odwf_status worst = ODWF_OK;
  for (int k0 = 0; k0 < nmass; k0 += per_launch) {
    const int n = std::min(per_launch, nmass - k0);
    if (use_y0)
      for (int q = 0; q < n; q++)
        HIPCHK(launch_vec_copy_rhs(PREC64, y, nullptr, nmass, k0 + q, PREC64, yg.d, nullptr, n, q, h, Ns, st));
    odwf_status sc = solve_chunk(S, ODWF_SOLVE_EO_NORMAL, mq + k0, tol + k0, 0, n, (int)inner, maxiter, b,
                                 nullptr, use_y0, stats ? stats + k0 : nullptr, st, io);
    if (sc == ODWF_EHIP || sc == ODWF_ENOMEM || sc == ODWF_EINVAL) return sc;
    if (sc != ODWF_OK && worst == ODWF_OK) worst = sc;
    for (int q = 0; q < n; q++)
      HIPCHK(launch_vec_copy_rhs(PREC64, yg.d, nullptr, n, q, PREC64, y, nullptr, nmass, k0 + q, h, Ns, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  return worst;
}

extern "C" odwf_status odwf_deff(odwf_solver S, int inverse, const double* mq, const double* tol, int nrhs,
                                 odwf_prec inner, int maxiter, const void* q, void* out,
                                 odwf_stats* stats, void* stream) {
  REQUIRE(S && mq && tol && q && out, "odwf_deff: null argument");
  REQUIRE(q != out, "odwf_deff: q and out must be distinct buffers");
  REQUIRE(nrhs >= 1, "odwf_deff: nrhs must be >= 1");
  REQUIRE(inner >= ODWF_FP64 && inner <= ODWF_BF16S, "odwf_deff: bad inner precision");
  REQUIRE(maxiter >= 1, "odwf_deff: maxiter must be >= 1");
  REQUIRE(S->lat->loaded, "odwf_deff: gauge field not loaded");
  for (int r = 0; r < nrhs; r++) {
    REQUIRE(std::isfinite(mq[r]), "odwf_deff: mq must be finite");
    REQUIRE(tol[r] > 0 && tol[r] < 1, "odwf_deff: tol must be in (0, 1)");
  }
  HIPCHK(hipSetDevice(S->lat->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lk(S->mtx);
  Workspace& W = S->workspace(st);
  const Geom& g = S->lat->g;
  const int Ns = S->Ns;
  const HalfFn get = [&](const char* name, int n, int p) { return W.half(name, g.h, n, Ns, p); };
  const int chunk = max_rhs_per_launch(Ns);
  const double mpv = 2.0 * S->m0;
  odwf_status worst = ODWF_OK;
  for (int r0 = 0; r0 < nrhs; r0 += chunk) {
    const int n = std::min(chunk, nrhs - r0);
    const size_t bytes5 = (size_t)n * Ns * g.V * 12 * 16;
    void* phi = W.get("d.phi", bytes5);
    void* psi = W.get("d.psi", bytes5);
    if (!phi || !psi) {
      set_error("odwf_deff: out of device memory for workspaces");
      return ODWF_ENOMEM;
    }
    // D_eff q = R D(m_PV)^{-1} D(m_q) R^T q;  D_eff^{-1} q = R D(m_q)^{-1} D(m_PV) R^T q
    double ma[MAXRHS], mb[MAXRHS];
    for (int k = 0; k < n; k++) {
      ma[k] = inverse ? mpv : mq[r0 + k];
      mb[k] = inverse ? mq[r0 + k] : mpv;
    }
    const size_t off4 = (size_t)r0 * g.V * 12 * 16;
    HIPCHK(launch_boundary_embed(static_cast<const char*>(q) + off4, phi, n, Ns, g, st));
    odwf_status sa = apply_chunk(S, ODWF_OP_D, ma, PREC64, 0, n, phi, psi, st, get, false);
    if (sa != ODWF_OK) return sa;
    odwf_status ss = solve_chunk(S, ODWF_SOLVE_FULL, mb, tol + r0, 0, n, (int)inner, maxiter, psi, phi, 0,
                                 stats ? stats + r0 : nullptr, st);
    if (ss == ODWF_EHIP || ss == ODWF_ENOMEM || ss == ODWF_EINVAL) return ss;
    if (ss != ODWF_OK && worst == ODWF_OK) worst = ss;
    HIPCHK(launch_boundary_project(phi, static_cast<char*>(out) + off4, n, Ns, g, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  return worst;
}

extern "C" odwf_status odwf_force(odwf_solver S, const void* chi, const void* psi, int accumulate,
                                  void* F, void* stream) {
  REQUIRE(S && chi && psi && F, "odwf_force: null argument");
  REQUIRE(F != chi && F != psi, "odwf_force: F must not alias chi or psi");
  REQUIRE(S->lat->loaded, "odwf_force: gauge field not loaded");
  HIPCHK(hipSetDevice(S->lat->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lk(S->mtx);
  Workspace& W = S->workspace(st);
  const Geom& g = S->lat->g;
  const int Ns = S->Ns;
  HV ce = W.half("f.ce", g.h, 1, Ns, PREC64), co = W.half("f.co", g.h, 1, Ns, PREC64);
  HV pe = W.half("f.pe", g.h, 1, Ns, PREC64), po = W.half("f.po", g.h, 1, Ns, PREC64);
  if (!ce.d || !co.d || !pe.d || !po.d) {
    set_error("odwf_force: out of device memory for workspaces");
    return ODWF_ENOMEM;
  }
  HIPCHK(launch_pack_spinor(PREC64, chi, 0, ce.d, nullptr, 0, 1, Ns, g, st));
  HIPCHK(launch_pack_spinor(PREC64, chi, 0, co.d, nullptr, 1, 1, Ns, g, st));
  HIPCHK(launch_pack_spinor(PREC64, psi, 0, pe.d, nullptr, 0, 1, Ns, g, st));
  HIPCHK(launch_pack_spinor(PREC64, psi, 0, po.d, nullptr, 1, 1, Ns, g, st));
  HIPCHK(launch_force(ce.d, pe.d, co.d, po.d, S->lat->U64[0], F, 0, Ns, S->lat->bc_t, accumulate, g, st));
  HIPCHK(launch_force(co.d, po.d, ce.d, pe.d, S->lat->U64[1], F, 1, Ns, S->lat->bc_t, accumulate, g, st));
  return ODWF_OK;
}

extern "C" odwf_status odwf_solver_reserve(odwf_solver S, int nrhs, odwf_prec inner, void* stream) {
  REQUIRE(S, "odwf_solver_reserve: null solver");
  REQUIRE(nrhs >= 1, "odwf_solver_reserve: nrhs must be >= 1");
  REQUIRE(inner >= ODWF_FP64 && inner <= ODWF_BF16S, "odwf_solver_reserve: bad inner precision");
  HIPCHK(hipSetDevice(S->lat->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lk(S->mtx);
  SolveBufs B;
  const int n = std::min(nrhs, max_rhs_per_launch(S->Ns));
  if (!solve_buffers(S->workspace(st), S->lat->g.h, n, S->Ns, (int)inner, B)) {
    set_error("odwf_solver_reserve: out of device memory");
    return ODWF_ENOMEM;
  }
  return ODWF_OK;
}

extern "C" odwf_status odwf_footprint(const int dims[4], int Ns, int nrhs, odwf_prec inner,
                                      size_t* bytes) {
  REQUIRE(dims && bytes, "odwf_footprint: null argument");
  REQUIRE(ns_supported(Ns) && nrhs >= 1, "odwf_footprint: bad Ns or nrhs");
  const long h = (long)dims[0] * dims[1] * dims[2] * dims[3] / 2;
  *bytes = solve_workspace_bytes(h, Ns, std::min(nrhs, max_rhs_per_launch(Ns)), (int)inner);
  return ODWF_OK;
}

// ------------------------------------------------------------------------------
// optimal weights
// ------------------------------------------------------------------------------

// Jacobi amplitude by the arithmetic-geometric mean and descending Landen
// transformation (Abramowitz & Stegun 16.4): returns dn(u | m) and K(m).
static void jacobi_dn_K(double u, double m, double* dn, double* K) {
  double a[64], c[64];
  a[0] = 1.0;
  double b = std::sqrt(1.0 - m);
  c[0] = std::sqrt(m);
  int n = 0;
  while (std::fabs(c[n]) > 1e-17 && n < 60) {
    a[n + 1] = 0.5 * (a[n] + b);
    c[n + 1] = 0.5 * (a[n] - b);
    b = std::sqrt(a[n] * b);
    n++;
  }
  *K = M_PI / (2.0 * a[n]);
  double phi = std::ldexp(1.0, n) * a[n] * u;
  double phi_prev = phi;
  for (int k = n; k >= 1; k--) {
    phi_prev = phi;
    phi = 0.5 * (phi + std::asin(c[k] / a[k] * std::sin(phi)));
  }
  // dn = cos(phi0) / cos(phi1 - phi0)
  *dn = n >= 1 ? std::cos(phi) / std::cos(phi_prev - phi) : 1.0;
}

extern "C" odwf_status odwf_zolotarev_omega(int Ns, double lmin, double lmax, double* omega) {
  REQUIRE(omega, "odwf_zolotarev_omega: null argument");
  REQUIRE(Ns >= 2 && Ns % 2 == 0, "odwf_zolotarev_omega: Ns must be even and >= 2");
  REQUIRE(lmin > 0 && lmax > lmin, "odwf_zolotarev_omega: need 0 < lambda_min < lambda_max");
  const double m = 1.0 - (lmin / lmax) * (lmin / lmax);
  double dn, K;
  jacobi_dn_K(0.0, m, &dn, &K);
  std::vector<double> half(Ns / 2);
  for (int k = 1; k <= Ns / 2; k++) {
    jacobi_dn_K((2 * k - 1) * K / Ns, m, &dn, &K);
    half[k - 1] = dn / lmin;
  }
  std::sort(half.begin(), half.end(), [](double p, double q) { return p > q; });
  for (int k = 0; k < Ns / 2; k++) {
    omega[k] = half[k];
    omega[Ns - 1 - k] = half[k];
  }
  return ODWF_OK;
}

// ------------------------------------------------------------------------------
// profiling and errors
// ------------------------------------------------------------------------------

extern "C" odwf_status odwf_profile_enable(int enable) {
  prof_enable(enable);
  return ODWF_OK;
}

extern "C" odwf_status odwf_profile_read(long long* launches, double* ms, double* bytes) {
  prof_read(launches, ms, bytes);
  return ODWF_OK;
}

extern "C" odwf_status odwf_profile_read_kernel(odwf_prec prec, int dag, long long* launches,
                                                double* ms, double* bytes) {
  REQUIRE(prec >= ODWF_FP64 && prec <= ODWF_BF16S, "odwf_profile_read_kernel: bad precision");
  prof_read_kernel((int)prec, dag, launches, ms, bytes);
  return ODWF_OK;
}

extern "C" const char* odwf_last_error(void) { return last_error_cstr(); }

extern "C" const char* odwf_version(void) { return "odwf-mi355x 0.1 (gfx950)"; }
