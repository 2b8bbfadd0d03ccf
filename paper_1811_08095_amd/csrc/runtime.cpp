// Host runtime: workspaces, fifth-dimension programs, kernel helpers and the
// hopping-kernel profiler.
#include "runtime.h"

#include <cstdio>
#include <cstdlib>
#include <cstring>

namespace odwf {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
const char* last_error_cstr() { return g_last_error.c_str(); }

size_t bytes_per_complex(int prec) {
  switch (prec) {
    case PREC64: return 16;
    case PREC32: return 8;
    default: return 4;
  }
}

size_t half_bytes(long h, int nrhs, int Ns, int prec) {
  return (size_t)h * nrhs * Ns * 12 * bytes_per_complex(prec);
}

size_t scale_bytes(long h, int nrhs, int Ns, int prec) {
  return (prec == PREC16 || prec == PRECB16) ? (size_t)h * nrhs * Ns * sizeof(float) : 0;
}

Workspace::~Workspace() {
  for (auto& kv : bufs)
    if (kv.second.p) (void)hipFree(kv.second.p);
}

void* Workspace::get(const std::string& name, size_t bytes) {
  if (bytes == 0) bytes = 16;
  DevBuf& b = bufs[name];
  if (b.bytes >= bytes) return b.p;
  if (b.p) {
    (void)hipDeviceSynchronize();
    (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
  }
  if (hipMalloc(&b.p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return nullptr;
  }
  b.bytes = bytes;
  return b.p;
}

HV Workspace::half(const std::string& name, long h, int nrhs, int Ns, int prec) {
  HV v;
  v.prec = prec;
  v.d = get(name, half_bytes(h, nrhs, Ns, prec));
  const size_t sb = scale_bytes(h, nrhs, Ns, prec);
  if (sb) v.sc = reinterpret_cast<float*>(get(name + ".sc", sb));
  return v;
}

size_t Workspace::total() const {
  size_t t = 0;
  for (auto& kv : bufs) t += kv.second.bytes;
  return t;
}

// ---- fifth-dimension programs -------------------------------------------------

static M5Prog mk(std::initializer_list<M5Op> ops) {
  M5Prog p;
  std::memset(&p, 0, sizeof(p));
  p.n = 0;
  for (const M5Op& o : ops) p.op[p.n++] = o;
  return p;
}
static M5Op op(M5Type t, CoefId d, CoefId e = CF_ONE) { return M5Op{t, d, e, 0}; }

M5Prog prog_none() { return mk({}); }
// A^{-1} = (1 + L) B^{-1} omega,  B = a + c L
M5Prog prog_ainv() {
  return mk({op(M5_SCALE, CF_OMEGA), op(M5_SOLVE_LO, CF_A_INV, CF_C), op(M5_MUL_LO, CF_ONE, CF_ONE)});
}
// A^{-T} = omega B^{-T} (1 + L)^T
M5Prog prog_ainv_t() {
  return mk({op(M5_MUL_UP, CF_ONE, CF_ONE), op(M5_SOLVE_UP, CF_A_INV, CF_CSHIFT), op(M5_SCALE, CF_OMEGA)});
}
// A = omega^{-1} B (1 + L)^{-1}
M5Prog prog_a() {
  return mk({op(M5_SOLVE_LO, CF_ONE, CF_ONE), op(M5_MUL_LO, CF_A, CF_C), op(M5_SCALE, CF_OMEGA_INV)});
}
// A^T = (1 + L)^{-T} B^T omega^{-1}
M5Prog prog_a_t() {
  return mk({op(M5_SCALE, CF_OMEGA_INV), op(M5_MUL_UP, CF_A, CF_CSHIFT), op(M5_SOLVE_UP, CF_ONE, CF_ONE)});
}
M5Prog prog_omega() { return mk({op(M5_SCALE, CF_OMEGA)}); }
M5Prog prog_omega_inv() { return mk({op(M5_SCALE, CF_OMEGA_INV)}); }
M5Prog prog_1pl() { return mk({op(M5_MUL_LO, CF_ONE, CF_ONE)}); }
M5Prog prog_1pl_inv() { return mk({op(M5_SOLVE_LO, CF_ONE, CF_ONE)}); }
M5Prog prog_1pl_t() { return mk({op(M5_MUL_UP, CF_ONE, CF_ONE)}); }

// ---- kernel helpers -------------------------------------------------------------

static size_t site_bytes(int prec) {
  return 12 * bytes_per_complex(prec) + ((prec == PREC16 || prec == PRECB16) ? 4 : 0);
}

// ---- block traversal of the hopping kernel -------------------------------------
// Default, when the x-rows split evenly into blocks: tiles of one x-row
// segment by 8 (4 when Ly is not a multiple of 8) by 4 rows in (y, z), t
// innermost, the eight XCDs walking a group of 4 x 2 adjacent tiles in
// lockstep (other group shapes, then contiguous XCD ranges, when the tile
// counts do not divide).  Otherwise XCD-aware contiguous block ranges.
// ODWF_TRAVERSAL ("linear", "xcd", "Ty,Tz", "Ty,Tz,Tt" or "Ty,Tz,Tt,Tx"; Tx = 0
// is the whole row) and ODWF_XCD ("contiguous", "lockstep" or "lockstep:Gy",
// Gy the tiles of a group along y) override for tuning.
static void traversal(HopArgs& a, int Ns) {
  const int inner = a.nrhs * Ns;
  const int spb = 256 / inner;
  const int hx = a.L[0] / 2;
  a.xcd = 1;
  a.tile_y = a.tile_z = a.tile_t = a.tile_x = 0;
  a.xcd_gy = 4;
  int ty = a.L[1] % 8 == 0 ? 8 : 4, tz = 4, tt = 0, tx = 1, gy = 4;
  bool lockstep = true;
  const char* env = getenv("ODWF_TRAVERSAL");
  if (env) {
    if (!strcmp(env, "linear")) {
      a.xcd = 0;
      return;
    }
    if (!strcmp(env, "xcd")) return;
    const int n = sscanf(env, "%d,%d,%d,%d", &ty, &tz, &tt, &tx);
    if (n < 2) return;
    if (n < 3) tt = 0;
    if (n < 4) tx = 0;
  }
  if (const char* xe = getenv("ODWF_XCD")) {
    lockstep = !strncmp(xe, "lockstep", 8);
    if (lockstep && xe[8] == ':') gy = atoi(xe + 9);
  }
  if (ty > 0 && tz > 0 && hx % spb == 0 && a.L[1] % ty == 0 && a.L[2] % tz == 0) {
    const int nseg = hx / spb;
    a.tile_y = ty;
    a.tile_z = tz;
    if (tt > 0 && a.L[3] % tt == 0) a.tile_t = tt;
    if (tx > 0 && nseg % tx == 0) a.tile_x = tx;
    if (lockstep) {
      const int nty = a.L[1] / ty, ntz = a.L[2] / tz;
      const int pref[5] = {gy, 4, 2, 8, 1};
      for (int g : pref) {
        if ((g == 1 || g == 2 || g == 4 || g == 8) && nty % g == 0 && ntz % (8 / g) == 0) {
          a.xcd = 2;
          a.xcd_gy = g;
          break;
        }
      }
    }
  }
}

hipError_t hop(const OpCtx& c, int out_par, int dag, const HV& in, const HV* out, const HopOpt& o) {
  HopArgs a;
  std::memset(&a, 0, sizeof(a));
  const odwf_lattice L = c.S->lat;
  a.in = in.d;
  a.in_sc = in.sc;
  a.links = c.links(out_par);
  a.out = out ? out->d : nullptr;
  a.out_sc = out ? out->sc : nullptr;
  a.xin = o.x ? o.x->d : nullptr;
  a.xin_sc = o.x ? o.x->sc : nullptr;
  a.cg_r = o.cg_r ? o.cg_r->d : nullptr;
  a.cg_r_sc = o.cg_r ? o.cg_r->sc : nullptr;
  a.cg_p = o.cg_p ? o.cg_p->d : nullptr;
  a.cg_p_sc = o.cg_p ? o.cg_p->sc : nullptr;
  a.scal = o.scal;
  a.partial = o.partial;
  a.gate = o.gate;
  a.gate_mode = o.gate ? o.gate_mode : GATE_NONE;
  a.coef = c.coef();
  for (int r = 0; r < MAXRHS; r++) a.kappa[r] = r < c.nrhs ? c.kappa[r] : 0.0;
  a.prog_h = o.ph;
  a.prog_x = o.px;
  a.prog_o = o.po;
  a.c_h = o.ch;
  a.c_x = o.cx;
  a.h = (int)L->g.h;
  a.nrhs = c.nrhs;
  a.out_par = out_par;
  a.bc_t = L->bc_t;
  a.dag = dag;
  for (int d = 0; d < 4; d++) a.L[d] = L->g.L[d];
  traversal(a, c.S->Ns);
  // launches gated to the active right-hand sides of a batch are counted with
  // the bytes of all nrhs (exact while every slot is active); launches gated to
  // pending reliable updates mostly exit at once and are not counted
  const bool prof = prof_on() && !c.noprof && (!o.gate || o.gate_mode == GATE_ACTIVE);
  if (prof) prof_begin(c.st, (c.prec & 3) * 2 + (dag ? 1 : 0));
  hipError_t e = launch_hop(a, c.prec, c.S->Ns, c.st);
  if (prof) {
    const double n5 = (double)L->g.h * c.nrhs * c.S->Ns;
    int streams = 1 + (out ? 1 : 0) + (o.x ? 1 : 0);
    if (o.cg_r) streams += 2;          // r read and written
    else if (o.cg_p) streams += 1;     // f read
    const double link_b = (double)L->g.h * 8 * (c.prec == PREC64 ? 18 * 8 : 12 * 4);
    prof_end(c.st, n5 * site_bytes(c.prec) * streams + link_b);
  }
  return e;
}

hipError_t m5(const OpCtx& c, const HV& in, const HV& out, const M5Prog& p, double c0,
              const HV* other, double c1) {
  KappaArr k;
  for (int r = 0; r < MAXRHS; r++) k.v[r] = r < c.nrhs ? c.kappa[r] : 0.0;
  return launch_m5(c.prec, in.d, in.sc, out.d, out.sc, other ? other->d : nullptr,
                   other ? other->sc : nullptr, c0, c1, p, c.coef(), k, c.h(), c.nrhs, c.Ns(), c.st);
}

// ---- profiler -------------------------------------------------------------------

struct ProfRec {
  hipEvent_t a, b;
  double bytes;
  int key;  // prec * 2 + dag
};
static std::mutex g_prof_mtx;
static bool g_prof = false;
static std::vector<ProfRec> g_recs;
static std::vector<hipEvent_t> g_pool;
static thread_local hipEvent_t g_open = nullptr;
static long long g_launches = 0;
static double g_ms = 0.0, g_bytes = 0.0;
static long long g_k_launches[8] = {0};
static double g_k_ms[8] = {0}, g_k_bytes[8] = {0};
static thread_local int g_open_key = 0;

bool prof_on() { return g_prof; }

static hipEvent_t take_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

static void drain_locked() {
  for (ProfRec& r : g_recs) {
    float ms = 0.f;
    (void)hipEventSynchronize(r.b);
    (void)hipEventElapsedTime(&ms, r.a, r.b);
    g_ms += ms;
    g_bytes += r.bytes;
    g_launches += 1;
    g_k_ms[r.key] += ms;
    g_k_bytes[r.key] += r.bytes;
    g_k_launches[r.key] += 1;
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
}

void prof_begin(hipStream_t st, int key) {
  std::lock_guard<std::mutex> lk(g_prof_mtx);
  if (g_recs.size() > 4096) drain_locked();
  g_open_key = key;
  g_open = take_event();
  (void)hipEventRecord(g_open, st);
}

void prof_end(hipStream_t st, double bytes) {
  std::lock_guard<std::mutex> lk(g_prof_mtx);
  hipEvent_t b = take_event();
  (void)hipEventRecord(b, st);
  g_recs.push_back(ProfRec{g_open, b, bytes, g_open_key});
  g_open = nullptr;
}

void prof_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof_mtx);
  drain_locked();
  g_prof = on != 0;
  g_launches = 0;
  g_ms = 0.0;
  g_bytes = 0.0;
  for (int k = 0; k < 8; k++) {
    g_k_launches[k] = 0;
    g_k_ms[k] = g_k_bytes[k] = 0.0;
  }
}

void prof_read(long long* launches, double* ms, double* bytes) {
  std::lock_guard<std::mutex> lk(g_prof_mtx);
  drain_locked();
  if (launches) *launches = g_launches;
  if (ms) *ms = g_ms;
  if (bytes) *bytes = g_bytes;
}

void prof_read_kernel(int prec, int dag, long long* launches, double* ms, double* bytes) {
  std::lock_guard<std::mutex> lk(g_prof_mtx);
  drain_locked();
  const int key = (prec & 3) * 2 + (dag ? 1 : 0);
  if (launches) *launches = g_k_launches[key];
  if (ms) *ms = g_k_ms[key];
  if (bytes) *bytes = g_k_bytes[key];
}

}  // namespace odwf

odwf::Workspace& odwf_solver_s::workspace(hipStream_t st) {
  auto it = ws.find(st);
  if (it != ws.end()) return *it->second;
  odwf::Workspace* w = new odwf::Workspace();
  ws[st] = w;
  return *w;
}
