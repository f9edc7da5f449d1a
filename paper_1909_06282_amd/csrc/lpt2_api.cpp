// Host side of the C ABI declared in include/lpt2.h: argument validation,
// the plan (workspace, twiddles, growth-table cache), the kernel sequences of
// each entry point, and per-kernel event timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "lpt2.h"
#include "kernels.hpp"

using namespace lpt2;

// Device memory of lpt2_displace_noalloc: the 16 workspace slots of one
// realisation, then room for the growth and radial tables when the plan has
// none cached at the requested a.  Every GPU that runs the library holds one
// copy until the process ends.  Host code never passes the name `scratch`
// to a kernel or a copy (on the host it is only a stand-in for the symbol):
// it uses the device address from hipGetSymbolAddress, kept per device in
// g_scratch_ptr.
constexpr size_t kScratchSlotBytes = LPT2_NOALLOC_SLOT_BYTES;
constexpr size_t kScratchTableBytes = LPT2_NOALLOC_TABLE_BYTES;
static __device__ __align__(256) char scratch[kScratchSlotBytes + kScratchTableBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

namespace {

thread_local std::string g_err;  // errors without a plan

struct Tables {
  double a = 0.0;
  bool unit = false;       // radial tables without the sqrt(P) shaping (density input)
  int cand = -1;           // AUTO configurations: the candidate D2 was built for (-1: provisional T1)
  double* d1n = nullptr;   // nk normalised D1 on the nodes
  double* d2n = nullptr;   // nk normalised D2 on the nodes
  double* radial = nullptr;  // TAB_COUNT x n2cnt
};

struct Grid {
  lpt2_config cfg;
  int count = 1;
  int n = 0;
  long m = 0, nnm = 0, n3 = 0, n2cnt = 0;
  Cosmo c;
  double amp = 0.0, lkmin = 0.0, lkmax = 0.0;
  void* tw = nullptr;
  int tiles[3] = {0, 0, 0};  // columns per block: y/x single passes, fused y pass, fused x pass (0 = default)
  int rfirst = 0;            // index of this grid's first realisation
  int bsub = 1;              // realisations transformed side by side (a batch)
  size_t ws_off = 0;         // this grid's batch region in the workspace
  hipStream_t st = nullptr;  // own stream when the plan holds several grids
  hipEvent_t join = nullptr;
  unsigned* tq = nullptr;    // tile tickets of the persistent column passes (16 words, zero between launches)
  std::vector<Tables> tables;
  std::vector<Tables> gr_tables;  // GR growth at a (for S_GR and the triangle ratios)
  std::vector<std::pair<double, int>> auto_choice;  // AUTO: (a, chosen candidate)
};

struct GraphEntry {
  double a;
  std::vector<const void*> ptrs;  // noise, psi1, psi2 of every realisation
  hipGraph_t graph;
  hipGraphExec_t exec;
};

struct ProfEntry {
  const char* name;
  long long launches;
  double ms;
  double bytes;
};

}  // namespace

struct lpt2_plan_s {
  std::vector<Grid> grids;
  std::vector<int> rgrid;  // realisation -> grid
  int prec = PREC_F64;
  size_t es = 8;           // bytes per real scalar
  char* ws = nullptr;
  size_t ws_bytes = 0;
  double* bin_partial = nullptr;
  double* bin_out = nullptr;
  unsigned long long* counter = nullptr;  // lpt2_check_finite (inside the binner allocation)
  std::string err;
  std::atomic<int> busy{0};
  bool prof = false;
  std::vector<ProfEntry> prof_tab;
  struct Pending { int idx; hipEvent_t a, b; };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  hipEvent_t fork = nullptr;        // several grids: their streams wait on this
  bool graph_mode = false;
  bool capturing = false;            // no per-launch events inside a capture
  bool quiet = false;                // no per-launch events (the allocation-free entry point)
  hipStream_t cap_stream = nullptr;  // stream the graphs are captured on
  std::vector<GraphEntry> graphs;
};

namespace {

constexpr int WS_FIELDS = 16;  // half-spectrum-sized slots in the workspace
constexpr size_t BATCH_WS_BUDGET = (size_t)16 << 30;  // workspace bytes a grid's batch may take

lpt2_status fail(lpt2_plan_t p, lpt2_status st, const std::string& msg) {
  if (p)
    p->err = msg;
  else
    g_err = msg;
  return st;
}

// Device allocations of the library.  For tests of the out-of-memory paths,
// LPT2_FAIL_ALLOC=k makes the k-th allocation counted from the start of the
// latest lpt2_plan call on this thread (1-based) fail as if the device were
// out of memory.
thread_local long g_alloc_count = 0;
hipError_t dev_malloc(void** ptr, size_t bytes) {
  ++g_alloc_count;
  if (const char* f = std::getenv("LPT2_FAIL_ALLOC")) {
    const long k = std::atol(f);
    if (k > 0 && g_alloc_count == k) {
      *ptr = nullptr;
      return hipErrorOutOfMemory;
    }
  }
  return hipMalloc(ptr, bytes);
}

lpt2_status hip_fail(lpt2_plan_t p, hipError_t e, const char* what) {
  return fail(p, LPT2_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Device address of `scratch` on the current device: resolved once per device
// (with that device current) and kept; later calls only look it up.
lpt2_status scratch_address(lpt2_plan_t p, char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(p, e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(p, LPT2_EDEVICE, "device index beyond the scratch address table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(p, e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(p, LPT2_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = ptr;
  }
  *out = (char*)g_scratch_ptr[dev];
  return LPT2_OK;
}

struct Busy {
  lpt2_plan_t p;
  bool ok;
  explicit Busy(lpt2_plan_t q) : p(q) {
    int z = 0;
    ok = p->busy.compare_exchange_strong(z, 1);
  }
  ~Busy() {
    if (ok) p->busy.store(0);
  }
};

// powers of two 8..512, three times a power of two 24..768, and the sizes
// with a factor 5 or 7: 40, 56, 200, 400, 600, 700 (the paper's boxes of
// 200-700 Mpc/h at one particle per Mpc/h, Sec. 3)
bool supported_n(int n) {
  const bool p2 = n > 0 && (n & (n - 1)) == 0, m = n % 3 == 0 && n > 0 && ((n / 3) & (n / 3 - 1)) == 0;
  const bool q = n == 40 || n == 56 || n == 200 || n == 400 || n == 600 || n == 700;
  return (p2 && n >= 8 && n <= 512) || (m && n >= 24 && n <= 768) || q;
}

// sigma8 normalisation: A = sigma8^2 / [(1/2 pi^2) Int k^3 k^ns T^2 W^2(8k) dln k],
// composite Simpson on ln k in [ln 1e-5, ln 1e3] with 2^16 intervals.
double sigma8_amplitude(const Cosmo& c, double sigma8) {
  const int nint = 1 << 16;
  const double lo = std::log(1e-5), hi = std::log(1e3), h = (hi - lo) / nint;
  auto f = [&](int i) {
    const double k = std::exp(lo + (hi - lo) * (double)i / (double)nint);
    const double t = bbks(c, k);
    const double x = 8.0 * k;
    const double w = 3.0 * (std::sin(x) - x * std::cos(x)) / (x * x * x);
    return k * k * k * std::pow(k, c.ns) * t * t * w * w / (2.0 * kPi * kPi);
  };
  double s = f(0) + f(nint), s4 = 0.0, s2 = 0.0;
  for (int i = 1; i < nint; i += 2) s4 += f(i);
  for (int i = 2; i < nint; i += 2) s2 += f(i);
  s += 4.0 * s4 + 2.0 * s2;
  return sigma8 * sigma8 / (s * h / 3.0);
}

lpt2_status validate(const lpt2_config& c, std::string& why) {
  if (!supported_n(c.n)) {
    why = "n must be a power of two in 8..512, three times one in 24..768, or one of 40, 56, 200, 400, 600, 700";
    return LPT2_EUNSUPPORTED;
  }
  if (c.precision != LPT2_FP64 && c.precision != LPT2_FP32) {
    why = "unknown precision";
    return LPT2_EUNSUPPORTED;
  }
  if (!(c.box > 0.0) || !std::isfinite(c.box)) { why = "box must be > 0"; return LPT2_EINVAL; }
  if (!(c.omega_m > 0.0 && c.omega_m <= 1.0)) { why = "omega_m must be in (0, 1]"; return LPT2_EINVAL; }
  if (!(c.h > 0.0) || !(c.sigma8 > 0.0) || !std::isfinite(c.n_s)) { why = "h, sigma8 must be > 0"; return LPT2_EINVAL; }
  if (c.gravity < 0 || c.gravity > 2) { why = "unknown gravity model"; return LPT2_EINVAL; }
  if (c.gravity == LPT2_GRAV_FR_HS) {
    if (!(c.fr0_abs > 0.0)) { why = "fr0_abs must be > 0 for f(R)"; return LPT2_EINVAL; }
    if (c.hs_n != 1) { why = "only Hu-Sawicki n = 1 has its M_k coefficients given"; return LPT2_EUNSUPPORTED; }
  }
  if (c.gravity == LPT2_GRAV_MU_CONST && !(c.mu_const > 0.0)) { why = "mu_const must be > 0"; return LPT2_EINVAL; }
  if (c.factorisation < 0 || c.factorisation > LPT2_D2_AUTO) { why = "unknown factorisation"; return LPT2_EINVAL; }
  if (c.factorisation == LPT2_D2_TRIANGLE &&
      (!(c.tri_ratio > 0.0) || !(c.tri_theta_deg > 0.0 && c.tri_theta_deg < 180.0))) {
    why = "triangle needs ratio > 0 and 0 < theta < 180";
    return LPT2_EINVAL;
  }
  if (c.nk_growth < 2 || c.nk_growth > 1023) { why = "nk_growth must be in 2..1023"; return LPT2_EINVAL; }
  if (!(c.kmin > 0.0) || !(c.kmax > c.kmin)) { why = "need 0 < kmin < kmax"; return LPT2_EINVAL; }
  if (!(c.a_init > 0.0 && c.a_init < 1.0)) { why = "a_init must be in (0, 1)"; return LPT2_EINVAL; }
  if (c.ode_steps < 1 || c.ode_steps > (1 << 24)) { why = "ode_steps must be in 1..2^24"; return LPT2_EINVAL; }
  return LPT2_OK;
}

double cos_deg(double th) { return th == 90.0 ? 0.0 : std::cos(th * kPi / 180.0); }

// ---- profiling ---------------------------------------------------------------
// one entry per (launch site, bytes per launch): the same site on grids or
// batches of different sizes is counted separately
int prof_slot(lpt2_plan_t p, const char* name, double bytes) {
  for (size_t i = 0; i < p->prof_tab.size(); ++i)
    if (p->prof_tab[i].name == name && p->prof_tab[i].bytes == bytes) return (int)i;
  p->prof_tab.push_back({name, 0, 0.0, bytes});
  return (int)p->prof_tab.size() - 1;
}
hipEvent_t take_event(lpt2_plan_t p) {
  if (!p->pool.empty()) {
    hipEvent_t e = p->pool.back();
    p->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
void prof_flush(lpt2_plan_t p) {
  for (auto& q : p->pending) {
    float ms = 0.f;
    if (hipEventSynchronize(q.b) == hipSuccess && hipEventElapsedTime(&ms, q.a, q.b) == hipSuccess)
      p->prof_tab[q.idx].ms += ms;
    p->pool.push_back(q.a);
    p->pool.push_back(q.b);
  }
  p->pending.clear();
}

// Runs one launch, recording an event pair around it in profiling mode.
template <class F>
lpt2_status run(lpt2_plan_t p, hipStream_t s, const char* name, double bytes, F&& launch) {
  hipEvent_t a = nullptr, b = nullptr;
  int idx = -1;
  const bool prof = p->prof && !p->capturing && !p->quiet;
  if (prof) {
    idx = prof_slot(p, name, bytes);
    a = take_event(p);
    b = take_event(p);
    if (a) (void)hipEventRecord(a, s);
  }
  hipError_t e = launch();
  if (e != hipSuccess) return hip_fail(p, e, name);
  if (prof && a && b) {
    (void)hipEventRecord(b, s);
    p->pending.push_back({idx, a, b});
    p->prof_tab[idx].launches++;
  }
  return LPT2_OK;
}
#define RUN(name, bytes, expr)                                              \
  do {                                                                      \
    lpt2_status st_ = run(p, s, name, (double)(bytes), [&]() { return (expr); }); \
    if (st_ != LPT2_OK) return st_;                                         \
  } while (0)

#define CHK(x)                      \
  do {                              \
    lpt2_status st_ = (x);          \
    if (st_ != LPT2_OK) return st_; \
  } while (0)

// Destroys the captured graphs (the caller has synchronised the device).
void drop_graphs(lpt2_plan_t p) {
  for (auto& ge : p->graphs) {
    if (ge.exec) (void)hipGraphExecDestroy(ge.exec);
    if (ge.graph) (void)hipGraphDestroy(ge.graph);
  }
  p->graphs.clear();
}

// ---- candidate triangles of the factorisation choice -----------------------------
// (Sec. 3, triangle comparison)
struct Candidate {
  const char* name;
  double ratio, theta;
  int winther;
};
const Candidate kCandidates[] = {
    {"T1", 1.0, 90.0, 0},        {"T2", 1.0, 80.0, 0},    {"iso70", 1.0, 70.0, 0}, {"equilateral", 1.0, 60.0, 0},
    {"squeezed", 1e-3, 90.0, 0}, {"r2_80", 2.0, 80.0, 0}, {"r2_70", 2.0, 70.0, 0}, {"winther", 1.0, 90.0, 1},
};
constexpr int kNCandidates = (int)(sizeof(kCandidates) / sizeof(kCandidates[0]));
constexpr int kAutoNone = -1;

int auto_lookup(const Grid& g, double a) {
  for (const auto& c : g.auto_choice)
    if (c.first == a) return c.second;
  return kAutoNone;
}

// ---- growth tables -------------------------------------------------------------
// Launches the growth-ODE and radial-table kernels of (a, gr, unit) into the
// memory t already points at: d1n, d2n (nk doubles each) and, unless gr,
// radial (TAB_ROWS x n2cnt doubles).  Allocates nothing.
lpt2_status build_tables_into(lpt2_plan_t p, Grid& g, double a, bool gr, bool unit, hipStream_t s, Tables& t) {
  const lpt2_config& cf = g.cfg;
  t.a = a;
  t.unit = unit;
  t.cand = kAutoNone;
  const int nk = cf.nk_growth;
  GrowthSetup gs;
  gs.c = g.c;
  if (gr) gs.c.gravity = GRAV_GR;
  gs.a_init = cf.a_init;
  gs.a = a;
  gs.steps = cf.ode_steps;
  gs.nk = nk;
  gs.lkmin = g.lkmin;
  gs.lkmax = g.lkmax;
  gs.winther = 0;
  gs.ratio = 1.0;
  gs.cs = 0.0;
  int fac = gr ? LPT2_D2_EDS : cf.factorisation;
  double tri_ratio = cf.tri_ratio, tri_theta = cf.tri_theta_deg;
  if (fac == LPT2_D2_AUTO) {  // the chosen candidate at a, else provisionally T1 (D1 does not depend on it)
    t.cand = auto_lookup(g, a);
    fac = LPT2_D2_T1;
    if (t.cand >= 0) {
      const Candidate& q = kCandidates[t.cand];
      fac = q.winther ? LPT2_D2_WINTHER : LPT2_D2_TRIANGLE;
      tri_ratio = q.ratio;
      tri_theta = q.theta;
    }
  }
  switch (fac) {
    case LPT2_D2_EDS: gs.mode = 0; break;
    case LPT2_D2_BOUCHET: gs.mode = 2; break;
    case LPT2_D2_TRIANGLE:
      gs.mode = 1;
      gs.ratio = tri_ratio;
      gs.cs = cos_deg(tri_theta);
      break;
    case LPT2_D2_WINTHER: gs.mode = 1; gs.winther = 1; break;
    default: gs.mode = 1; break;  // T1
  }
  CHK(run(p, s, "growth_ode", 0.0, [&]() { return launch_growth(gs, t.d1n, t.d2n, s); }));
  if (!gr) {
    RadialSetup rs;
    rs.c = g.c;
    rs.n = g.n;
    rs.box = cf.box;
    rs.amp = g.amp;
    rs.a = a;
    rs.nk = nk;
    rs.lkmin = g.lkmin;
    rs.lkmax = g.lkmax;
    rs.unit = unit ? 1 : 0;
    CHK(run(p, s, "radial_tables", 0.0, [&]() { return launch_radial(rs, t.d1n, t.d2n, t.radial, g.n2cnt, s); }));
  }
  return LPT2_OK;
}

lpt2_status build_tables(lpt2_plan_t p, Grid& g, double a, bool gr, bool unit, hipStream_t s, Tables& out) {
  Tables t;
  const int nk = g.cfg.nk_growth;
  hipError_t e = dev_malloc((void**)&t.d1n, sizeof(double) * nk * 2);
  if (e != hipSuccess) return fail(p, LPT2_ENOMEM, "growth table allocation failed");
  t.d2n = t.d1n + nk;
  if (!gr) {
    e = dev_malloc((void**)&t.radial, sizeof(double) * TAB_ROWS * g.n2cnt);
    if (e != hipSuccess) {
      (void)hipFree(t.d1n);
      return fail(p, LPT2_ENOMEM, "radial table allocation failed");
    }
  }
  lpt2_status st = build_tables_into(p, g, a, gr, unit, s, t);
  if (st != LPT2_OK) {
    (void)hipFree(t.d1n);
    if (t.radial) (void)hipFree(t.radial);
    return st;
  }
  out = t;
  return LPT2_OK;
}

void free_tables(Tables& t) {
  (void)hipFree(t.d1n);
  if (t.radial) (void)hipFree(t.radial);
}

// the cached tables of (a, unit) that are current (for AUTO: built for the
// candidate chosen at a), or nullptr; no side effects
const Tables* find_tables(const Grid& g, double a, bool unit) {
  const int cand = g.cfg.factorisation == LPT2_D2_AUTO ? auto_lookup(g, a) : kAutoNone;
  for (const Tables& t : g.tables)
    if (t.a == a && t.unit == unit && t.cand == cand) return &t;
  return nullptr;
}

lpt2_status get_tables(lpt2_plan_t p, Grid& g, double a, bool gr, hipStream_t s, Tables** out, bool unit = false) {
  std::vector<Tables>& cache = gr ? g.gr_tables : g.tables;
  const int cand = (!gr && g.cfg.factorisation == LPT2_D2_AUTO) ? auto_lookup(g, a) : kAutoNone;
  for (size_t i = 0; i < cache.size(); ++i) {
    Tables& t = cache[i];
    if (t.a != a || t.unit != unit) continue;
    if (t.cand == cand) {
      *out = &t;
      return LPT2_OK;
    }
    // an AUTO configuration whose choice at a was made after these tables
    (void)hipStreamSynchronize(s);
    (void)hipDeviceSynchronize();
    drop_graphs(p);
    free_tables(t);
    cache.erase(cache.begin() + (long)i);
    break;
  }
  if (cache.size() >= 32) {  // drop the oldest entry once its users are done
    (void)hipStreamSynchronize(s);
    (void)hipDeviceSynchronize();
    drop_graphs(p);           // captured graphs may read the tables
    free_tables(cache.front());
    cache.erase(cache.begin());
  }
  Tables t;
  lpt2_status st = build_tables(p, g, a, gr, unit, s, t);
  if (st != LPT2_OK) return st;
  cache.push_back(t);
  *out = &cache.back();
  return LPT2_OK;
}

// ---- x-pass operators ---------------------------------------------------------
const int PI_[6] = {0, 1, 2, 0, 0, 1}, PJ_[6] = {0, 1, 2, 1, 2, 2};

XOp op_blank(int nin, int nout, int inverse) {
  XOp op;
  std::memset(&op, 0, sizeof(op));
  op.nin = nin;
  op.nout = nout;
  op.inverse = inverse;
  for (int i = 0; i < XOP_MAX; ++i) {
    op.ci[i] = op.cj[i] = op.table[i] = -1;
    op.scale[i] = 1.0;
    op.kind[i] = MUL_REAL;
  }
  return op;
}
void op_set(XOp& op, int c, int kind, int ci, int cj, int table, double scale) {
  op.kind[c] = kind;
  op.ci[c] = ci;
  op.cj[c] = cj;
  op.table[c] = table;
  op.scale[c] = scale;
}
void op_tables(XOp& op, const Grid& g, const Tables* t) {
  for (int i = 0; i < TAB_COUNT; ++i) op.tables[i] = t->radial + (long)i * g.n2cnt;
}

// ---- pipeline pieces ------------------------------------------------------------
// Workspace slot i holds one half spectrum (n*n*(n/2) complex = one real
// n^3 field) of each of the nr realisations of a batch, one after the other.
// Every launch passes the capacity of each buffer: for a slot, the bytes to
// the end of the workspace; for a caller's field, its documented size.
struct Ctx {
  lpt2_plan_t p;
  Grid& g;
  hipStream_t s;
  size_t cs;         // bytes per complex
  char* base;        // slot 0
  int nr = 1;        // realisations per slot
  char* end = nullptr;  // end of the workspace region this context may use (nullptr: the workspace end)
  char* lo = nullptr;   // start of that region (nullptr: the workspace start)
  long sstride() const { return (long)nr * g.nnm; }  // complex from one slot to the next
  char* slot(int i) const { return base + (size_t)i * sstride() * cs; }
  size_t cap(const void* ptr) const {  // bytes from a workspace pointer to the region end
    const char* q = (const char*)ptr;
    const char* b = lo ? lo : p->ws;
    const char* e = end ? end : p->ws + p->ws_bytes;
    return (q >= b && q < e) ? (size_t)(e - q) : 0;
  }
  size_t field() const { return (size_t)g.n3 * p->es; }  // bytes of one real field
  double fields(double k) const { return k * (double)field() * nr; }  // bytes of k fields of the batch
  // nf caller fields per realisation (n^3 reals apart) <-> nf slots from `ws`
  Batch batch(const void* const* ext, int nf) const {
    Batch b;
    std::memset(&b, 0, sizeof(b));
    b.nf = nf;
    b.nr = nr;
    b.ext_fstride = g.n3;
    b.ws_fstride = sstride();
    b.ws_rstride = g.nnm;
    for (int r = 0; r < nr; ++r) b.ext[r] = ext[r];
    return b;
  }
  Batch one(const void* ext, int nf) const { return batch_one(ext, nf, g.n3, sstride()); }
};

// forward z and y passes of `b` (caller fields, ext_cap bytes each) into spectral slots at `out`
lpt2_status fwd_zy(Ctx& c, const char* nz, const char* ny, const Batch& b, size_t ext_cap, void* out) {
  lpt2_plan_t p = c.p;
  hipStream_t s = c.s;
  Grid& g = c.g;
  const double by = 2.0 * (double)c.field() * b.nf * b.nr;
  RUN(nz, by, launch_zr2c(p->prec, g.n, b, ext_cap, out, c.cap(out), g.tw, s));
  RUN(ny, by,
      launch_colfft(p->prec, g.n, -1, out, c.cap(out), (long)b.nf * b.nr * g.n, g.n * g.m, (int)g.m, g.m, g.tw, s,
                    g.tiles[0]));
  return LPT2_OK;
}
lpt2_status inv_y(Ctx& c, const char* ny, void* data, int nf) {
  lpt2_plan_t p = c.p;
  hipStream_t s = c.s;
  Grid& g = c.g;
  RUN(ny, c.fields(2.0 * nf),
      launch_colfft(p->prec, g.n, +1, data, c.cap(data), (long)nf * c.nr * g.n, g.n * g.m, (int)g.m, g.m, g.tw, s,
                    g.tiles[0]));
  return LPT2_OK;
}
lpt2_status fwd_y(Ctx& c, const char* ny, void* data, int nf) {
  lpt2_plan_t p = c.p;
  hipStream_t s = c.s;
  Grid& g = c.g;
  RUN(ny, c.fields(2.0 * nf),
      launch_colfft(p->prec, g.n, -1, data, c.cap(data), (long)nf * c.nr * g.n, g.n * g.m, (int)g.m, g.m, g.tw, s,
                    g.tiles[0]));
  return LPT2_OK;
}
// generic x pass (one realisation per Ctx)
lpt2_status xp(Ctx& c, const char* name, const void* in, void* out, const XOp& op) {
  lpt2_plan_t p = c.p;
  hipStream_t s = c.s;
  Grid& g = c.g;
  if (c.nr != 1) return fail(p, LPT2_EINVAL, "generic x pass takes one realisation");
  const long fst = c.sstride();
  RUN(name, c.fields(op.nin + op.nout),
      launch_xpass(p->prec, g.n, in, c.cap(in), fst, out, c.cap(out), fst, op, g.n2cnt, g.tw, s));
  return LPT2_OK;
}
lpt2_status xdisp(Ctx& c, const char* name, int mode, const void* in, void* out, const Tables* t) {
  lpt2_plan_t p = c.p;
  hipStream_t s = c.s;
  Grid& g = c.g;
  const bool f32 = p->prec == PREC_F32;
  const int row = mode != 1 ? (f32 ? TAB_PAIR32 : TAB_PAIR64) : (f32 ? TAB_PSI2_32 : TAB_PSI2);
  const void* tab = t->radial + (size_t)row * g.n2cnt;
  const size_t cap = sizeof(double) * (size_t)(TAB_ROWS - row) * g.n2cnt;
  RUN(name, c.fields(mode == 0 ? 6 : (mode == 3 ? 4 : 3)),
      launch_xdisp(p->prec, g.n, c.nr, mode, in, c.cap(in), out, c.cap(out), c.sstride(), tab, cap, g.tw, s,
                   g.tiles[2], g.tq));
  return LPT2_OK;
}
// inverse z pass of nf slots at `in` into the fields of `b` (m_z powers rpow per field)
lpt2_status z_c2r(Ctx& c, const char* name, const void* in, const Batch& b, size_t ext_cap, const int* rpow = nullptr) {
  lpt2_plan_t p = c.p;
  hipStream_t s = c.s;
  Grid& g = c.g;
  ZPow zp = zpow_none();
  if (rpow)
    for (int f = 0; f < b.nf && f < ZPOW_MAX; ++f) zp.r[f] = rpow[f];
  RUN(name, 2.0 * (double)c.field() * b.nf * b.nr,
      launch_zc2r(p->prec, g.n, in, c.cap(in), b, ext_cap, zp, g.tw, s));
  return LPT2_OK;
}
// in-place inverse z pass of nf workspace slots (one realisation)
lpt2_status z_c2r_ws(Ctx& c, const char* name, void* data, int nf) {
  return z_c2r(c, name, data, c.one(data, nf), c.cap(data));
}
lpt2_status z_source(Ctx& c, const void* phi, void* sk, const int* rpow = nullptr, const int* fmap = nullptr) {
  lpt2_plan_t p = c.p;
  hipStream_t s = c.s;
  Grid& g = c.g;
  ZPow zp = zpow_none();
  for (int f = 0; f < 6; ++f) {
    if (rpow) zp.r[f] = rpow[f];
    if (fmap) zp.fmap[f] = fmap[f];
  }
  RUN("z_fused_source", c.fields(7.0),
      launch_zsource(p->prec, g.n, phi, c.cap(phi), c.sstride(), zp, sk, c.cap(sk), (long)c.nr * g.n * g.n, g.tw,
                     s));
  return LPT2_OK;
}
lpt2_status ycombo(Ctx& c, const char* name, const void* in, void* out, const YOp& op) {
  lpt2_plan_t p = c.p;
  hipStream_t s = c.s;
  Grid& g = c.g;
  RUN(name, c.fields(op.nin + op.nout),
      launch_ycombo(p->prec, g.n, c.nr, in, c.cap(in), c.sstride(), out, c.cap(out), c.sstride(), op, g.tw, s,
                    g.tiles[1], g.tq));
  return LPT2_OK;
}
YOp yop(int nin, int nout, const int* src, const int* pw) {
  YOp op;
  std::memset(&op, 0, sizeof(op));
  op.nin = nin;
  op.nout = nout;
  for (int o = 0; o < nout; ++o) {
    op.src[o] = src[o];
    op.pw[o] = pw[o];
  }
  return op;
}

// psi1, psi2 of the c.nr realisations of a batch (see lpt2_displace).  The
// k-space factors are split by axis: the radial part (and k_x) is applied in
// the x pass, k_y in the y pass and k_z in the z pass, so five x-transforms
// carry the nine fields:  U_p = F_x^-1[-k_x^p A/k^2 X] (p = 0,1,2),
// V_p = F_x^-1[i k_x^p A D1/k^2 X] (p = 0,1), and e.g.
// phi_yz = F_z^-1[k_z F_y^-1[k_y U_0]] (integer mode numbers throughout;
// the (2 pi/L) factors sit in the radial tables).  Slots 0..15; on return
// slot 0 still holds F_zy[w] and slot 15 F_zy[S] (for further epochs).
lpt2_status displace_batch(Ctx& c, const Tables* t, const void* const* noise, void* const* psi1, void* const* psi2) {
  CHK(fwd_zy(c, "z_r2c_noise", "y_fwd_noise", c.batch(noise, 1), c.field(), c.slot(0)));
  CHK(xdisp(c, "x_fused_psi1_phi", 0, c.slot(0), c.slot(1), t));
  // outputs (inputs U0,U1,U2,V0,V1 = 0..4, grouped so each is read once):
  // psi1 x,y,z, then phi stored as xx,xy,xz,yy,zz,yz
  const int src9[9] = {4, 3, 3, 2, 1, 1, 0, 0, 0};
  const int pw9[9] = {0, 1, 0, 0, 1, 0, 2, 0, 1};
  CHK(ycombo(c, "y_inv_psi1_phi", c.slot(1), c.slot(6), yop(5, 9, src9, pw9)));
  const int rz1[3] = {0, 0, 1};
  CHK(z_c2r(c, "z_c2r_psi1", c.slot(6), c.batch(psi1, 3), 3 * c.field(), rz1));
  // source pass order xx,yy,zz,xy,xz,yz: m_z powers and storage positions
  const int rzs[6] = {0, 0, 2, 0, 1, 1};
  const int fms[6] = {0, 3, 4, 1, 2, 5};
  CHK(z_source(c, c.slot(9), c.slot(15), rzs, fms));
  CHK(fwd_y(c, "y_fwd_source", c.slot(15), 1));
  CHK(xdisp(c, "x_fused_psi2", 1, c.slot(15), c.slot(1), t));
  const int src3[3] = {1, 0, 0};
  const int pw3[3] = {0, 1, 0};
  CHK(ycombo(c, "y_inv_psi2", c.slot(1), c.slot(3), yop(2, 3, src3, pw3)));
  CHK(z_c2r(c, "z_c2r_psi2", c.slot(3), c.batch(psi2, 3), 3 * c.field(), rz1));
  return LPT2_OK;
}

// A further epoch of the batch whose displace_batch ran last on this context:
// psi1 and psi2 at the a of `t` from F_zy[w] (slot 0) and F_zy[S] (slot 15),
// which do not depend on a (the unevolved potential; Sec. 2.4 factorisation).
lpt2_status epoch_batch(Ctx& c, const Tables* t, void* const* psi1, void* const* psi2) {
  const int src3[3] = {1, 0, 0};  // V0, V1 (or Q0, Q1) -> x, y, z components
  const int pw3[3] = {0, 1, 0};
  const int rz1[3] = {0, 0, 1};
  CHK(xdisp(c, "x_psi1_epoch", 2, c.slot(0), c.slot(1), t));
  CHK(ycombo(c, "y_inv_psi1_epoch", c.slot(1), c.slot(3), yop(2, 3, src3, pw3)));
  CHK(z_c2r(c, "z_c2r_psi1", c.slot(3), c.batch(psi1, 3), 3 * c.field(), rz1));
  CHK(xdisp(c, "x_fused_psi2", 1, c.slot(15), c.slot(1), t));
  CHK(ycombo(c, "y_inv_psi2", c.slot(1), c.slot(3), yop(2, 3, src3, pw3)));
  CHK(z_c2r(c, "z_c2r_psi2", c.slot(3), c.batch(psi2, 3), 3 * c.field(), rz1));
  return LPT2_OK;
}

// S(k) of the displacement path, k-space, masked, times `scale`, into slot
// `dst` (uses slots 0..6 and 10)
lpt2_status source_k(Ctx& c, const Tables* t, const void* noise, int dst, double scale) {
  Grid& g = c.g;
  CHK(fwd_zy(c, "z_r2c_noise", "y_fwd_noise", c.one(noise, 1), c.field(), c.slot(0)));
  XOp op = op_blank(1, 6, 1);
  op_tables(op, g, t);
  for (int q = 0; q < 6; ++q) op_set(op, q, MUL_REAL, PI_[q], PJ_[q], TAB_PHI, -1.0);
  CHK(xp(c, "x_fused_phi", c.slot(0), c.slot(1), op));
  CHK(inv_y(c, "y_inv_phi", c.slot(1), 6));
  CHK(z_source(c, c.slot(1), c.slot(10)));
  CHK(fwd_y(c, "y_fwd_source", c.slot(10), 1));
  XOp o = op_blank(1, 1, 0);
  op_set(o, 0, MUL_REAL, -1, -1, -1, scale);
  CHK(xp(c, "x_fwd_source", c.slot(10), c.slot(dst), o));
  return LPT2_OK;
}

// S_MG(k) = S1+S2+S3+S4 into slot 10 (uses slots 0..10 and 12..15; slot 11
// is left alone).  The pairs (i,j) go in two groups, the diagonal ones and
// the others: one x pass gives each pair's fields R1, R2 (and R4) with the
// full k factors, one y pass inverts them, and one z pass (k_zmg) inverts
// them along z and accumulates the products in registers into real fields in
// slots 12..15: R1 (G S1 part), R2 + (tr phi)^2 (the C2 parts), R5 and chi^2.
lpt2_status mg_source_k(Ctx& c, const Tables* t, const void* noise) {
  lpt2_plan_t p = c.p;
  hipStream_t s = c.s;
  Grid& g = c.g;
  const bool fr = g.c.gravity == GRAV_FR;
  const int nt = fr ? 3 : 2;  // fields per pair
  if (c.cap(c.slot(12)) < 4 * c.field()) return fail(p, LPT2_EINVAL, "workspace too small");
  CHK(fwd_zy(c, "z_r2c_noise", "y_fwd_noise", c.one(noise, 1), c.field(), c.slot(0)));
  const long nlines = (long)g.n * g.n;
  const long afs = 2 * c.sstride();  // reals from one accumulator field to the next
  for (int grp = 0; grp < 2; ++grp) {
    XOp op = op_blank(1, 3 * nt, 1);
    op_tables(op, g, t);
    for (int k = 0; k < 3; ++k) {
      const int q = 3 * grp + k, i = PI_[q], j = PJ_[q];
      op_set(op, nt * k, MUL_REAL, i, j, TAB_R1, -1.0);
      op_set(op, nt * k + 1, MUL_REAL, i, j, TAB_R2, -1.0);
      if (fr) op_set(op, nt * k + 2, MUL_REAL, i, j, TAB_R4, -1.0);
    }
    CHK(xp(c, "x_mg_phi", c.slot(0), c.slot(1), op));
    CHK(inv_y(c, "y_inv_mg", c.slot(1), op.nout));
    RUN("z_mg_pairs", c.fields(op.nout + (grp == 0 ? nt : 2.0 * nt)),
        launch_zmg(p->prec, g.n, grp, nt, c.slot(1), c.cap(c.slot(1)), c.sstride(), c.slot(12), c.cap(c.slot(12)),
                   afs, nlines, g.tw, s));
  }
  if (fr) {
    XOp op = op_blank(1, 7, 1);
    op_tables(op, g, t);
    for (int j = 0; j < 3; ++j) {
      op_set(op, 2 * j, MUL_MI, j, -1, TAB_R5, 1.0);
      op_set(op, 2 * j + 1, MUL_PI, j, -1, TAB_R6, 1.0);
    }
    op_set(op, 6, MUL_REAL, -1, -1, TAB_R3, 1.0);
    CHK(xp(c, "x_mg_grad", c.slot(0), c.slot(1), op));
    CHK(inv_y(c, "y_inv_mg", c.slot(1), 7));
    RUN("z_mg_grad", c.fields(7.0 + 3.0),
        launch_zmg(p->prec, g.n, 2, 3, c.slot(1), c.cap(c.slot(1)), c.sstride(), c.slot(12), c.cap(c.slot(12)), afs,
                   nlines, g.tw, s));
  }
  const int nr = fr ? 4 : 2;
  CHK(fwd_zy(c, "z_r2c_mg", "y_fwd_mg", c.one(c.slot(12), nr), c.cap(c.slot(12)), c.slot(12)));
  const double G = four_pi_g_rho(g.c, t->a);
  XOp op = op_blank(nr, 1, 0);
  op_tables(op, g, t);
  op_set(op, 0, MUL_REAL, -1, -1, -1, G);        // F R1
  op_set(op, 1, MUL_REAL, -1, -1, TAB_C2, 1.0);  // F [R2 + (tr phi)^2]
  if (fr) {
    op_set(op, 2, MUL_REAL, -1, -1, TAB_C5, 1.0);  // F R5
    op_set(op, 3, MUL_REAL, -1, -1, TAB_C4, 1.0);  // F chi^2
  }
  CHK(xp(c, "x_fwd_mg", c.slot(12), c.slot(10), op));
  return LPT2_OK;
}

// adjoint x pass (mode 0: five inputs, the noise gradient; mode 1: two, S_bar), one realisation
lpt2_status xadj(Ctx& c, const char* name, int mode, const void* in, void* out, const Tables* t) {
  lpt2_plan_t p = c.p;
  hipStream_t s = c.s;
  Grid& g = c.g;
  if (c.nr != 1) return fail(p, LPT2_EINVAL, "adjoint x pass takes one realisation");
  const bool f32 = p->prec == PREC_F32;
  const int row = mode == 0 ? (f32 ? TAB_PAIR32 : TAB_PAIR64) : (f32 ? TAB_PSI2_32 : TAB_PSI2);
  const void* tab = t->radial + (size_t)row * g.n2cnt;
  const size_t cap = sizeof(double) * (size_t)(TAB_ROWS - row) * g.n2cnt;
  RUN(name, c.fields(mode == 0 ? 6 : 3),
      launch_xadj(p->prec, g.n, mode, in, c.cap(in), c.sstride(), out, c.cap(out), tab, cap, g.tw, s, g.tiles[2],
                  g.tq));
  return LPT2_OK;
}
// fan-in y pass over the c.nr realisations of each of op.nin slots at `in`
lpt2_status yfan(Ctx& c, const char* name, const void* in, void* out, const YFan& op) {
  lpt2_plan_t p = c.p;
  hipStream_t s = c.s;
  Grid& g = c.g;
  RUN(name, c.fields(op.nterm + op.nout),
      launch_yfanin(p->prec, g.n, c.nr, in, c.cap(in), c.sstride(), out, c.cap(out), c.sstride(), op, g.tw, s,
                    g.tiles[1], g.tq));
  return LPT2_OK;
}
// terms (src, m_y power, m_z power) of the outputs one after the other, nper[o] for output o
YFan yfan_op(int nin, int nout, const int* nper, const int (*terms)[3]) {
  YFan op;
  std::memset(&op, 0, sizeof(op));
  op.nin = nin;
  op.nout = nout;
  int k = 0;
  for (int o = 0; o < nout; ++o) {
    op.first[o] = k;
    for (int j = 0; j < nper[o]; ++j, ++k) {
      op.src[k] = terms[k][0];
      op.py[k] = terms[k][1];
      op.pz[k] = terms[k][2];
    }
  }
  op.first[nout] = k;
  op.nterm = k;
  return op;
}

// Gradient of a loss with respect to the noise of one realisation, from the
// gradients psi1_bar, psi2_bar of its displacements (the transpose of the
// linear maps of displace_batch, with S linearised about the noise).  The
// axis split of the forward chain runs backwards: z and y passes take the
// m_z, m_y powers and sum the fields that share a k_x power, so the x passes
// see one field per power.
//   S_bar = F^-1[i PSI2 (F_x Q0 + m_x F_x Q1)],
//     Q0 = m_y F_zy psi2_bar_y + m_z F_zy psi2_bar_z, Q1 = F_zy psi2_bar_x;
//   phi_bar_ij from S_bar and phi (product rule of S), phi by the forward split;
//   w_bar = F^-1[-PHI sum_p m_x^p F_x Ubar_p - i PSI1 sum_p m_x^p F_x Vbar_p],
//     Ubar_p, Vbar_p: the phi_bar_ij, psi1_bar_i of k_x power p, each times
//     its m_y, m_z powers after F_zy.
// Slots 0..14 of one realisation.
lpt2_status backward_one(Ctx& c, const Tables* t, const void* noise, const void* g1, const void* g2, void* gw) {
  lpt2_plan_t p = c.p;
  hipStream_t s = c.s;
  Grid& g = c.g;
  const double fb = (double)c.field();
  // S_bar into slot 10 (real)
  RUN("z_r2c_gpsi2", 2.0 * fb * 3,
      launch_zr2c(p->prec, g.n, c.one(g2, 3), 3 * c.field(), c.slot(1), c.cap(c.slot(1)), g.tw, s));
  const int nq[2] = {2, 1};
  const int tq[3][3] = {{1, 1, 0}, {2, 0, 1}, {0, 0, 0}};  // Q0: y, z; Q1: x
  CHK(yfan(c, "y_fan_gpsi2", c.slot(1), c.slot(4), yfan_op(3, 2, nq, tq)));
  CHK(xadj(c, "x_adj_psi2", 1, c.slot(4), c.slot(10), t));
  CHK(inv_y(c, "y_inv_sbar", c.slot(10), 1));
  CHK(z_c2r_ws(c, "z_c2r_sbar", c.slot(10), 1));
  // phi recomputed from the noise: U_p (slots 1..3), then phi stored as
  // xx,xy,xz,yy,zz,yz in slots 4..9; phi_bar overwrites it there
  CHK(fwd_zy(c, "z_r2c_noise", "y_fwd_noise", c.one(noise, 1), c.field(), c.slot(0)));
  CHK(xdisp(c, "x_phi_adj", 3, c.slot(0), c.slot(1), t));
  const int src6[6] = {2, 1, 1, 0, 0, 0};
  const int pw6[6] = {0, 1, 0, 2, 0, 1};
  CHK(ycombo(c, "y_inv_phi_adj", c.slot(1), c.slot(4), yop(3, 6, src6, pw6)));
  // product-rule pass order xx,yy,zz,xy,xz,yz: m_z powers and storage positions
  ZPow zp = zpow_none();
  const int rzs[6] = {0, 0, 2, 0, 1, 1};
  const int fms[6] = {0, 3, 4, 1, 2, 5};
  for (int f = 0; f < 6; ++f) {
    zp.r[f] = rzs[f];
    zp.fmap[f] = fms[f];
  }
  RUN("z_adj_prodrule", fb * 13.0,
      launch_zprodrule(p->prec, g.n, c.slot(4), c.cap(c.slot(4)), g.nnm, c.slot(10), c.cap(c.slot(10)), c.slot(4),
                       c.cap(c.slot(4)), g.nnm, (long)g.n * g.n, zp, g.tw, s));
  RUN("z_r2c_gpsi1", 2.0 * fb * 3,
      launch_zr2c(p->prec, g.n, c.one(g1, 3), 3 * c.field(), c.slot(1), c.cap(c.slot(1)), g.tw, s));
  // slots 1..9: psi1_bar x,y,z, phi_bar xx,xy,xz,yy,zz,yz -> Ubar0..2, Vbar0..1 in slots 10..14
  const int nu[5] = {3, 2, 1, 2, 1};
  const int tu[9][3] = {{6, 2, 0}, {7, 0, 2}, {8, 1, 1},  // Ubar0: yy, zz, yz
                        {4, 1, 0}, {5, 0, 1},             // Ubar1: xy, xz
                        {3, 0, 0},                        // Ubar2: xx
                        {1, 1, 0}, {2, 0, 1},             // Vbar0: psi1 y, z
                        {0, 0, 0}};                       // Vbar1: psi1 x
  CHK(yfan(c, "y_fan_adj", c.slot(1), c.slot(10), yfan_op(9, 5, nu, tu)));
  CHK(xadj(c, "x_adj_noise", 0, c.slot(10), c.slot(0), t));
  CHK(inv_y(c, "y_inv_gnoise", c.slot(0), 1));
  CHK(z_c2r(c, "z_c2r_gnoise", c.slot(0), c.one(gw, 1), c.field()));
  return LPT2_OK;
}

lpt2_status check_a(lpt2_plan_t p, double a) {
  if (!(a > 0.0) || !std::isfinite(a)) return fail(p, LPT2_EINVAL, "scale factor a must be > 0");
  return LPT2_OK;
}

// ---- batched displacement: grids, batches, streams, graphs -------------------------
// growth tables of every grid at a (built on s if missing)
lpt2_status tables_for(lpt2_plan_t p, double a, hipStream_t s, std::vector<Tables*>& out) {
  out.assign(p->grids.size(), nullptr);
  for (size_t i = 0; i < p->grids.size(); ++i) CHK(get_tables(p, p->grids[i], a, false, s, &out[i]));
  return LPT2_OK;
}

// every realisation of grid gi, bsub at a time, on `st`
lpt2_status run_grid(lpt2_plan_t p, int gi, const Tables* t, const void* const* noise, void* const* psi1,
                     void* const* psi2, hipStream_t st) {
  Grid& g = p->grids[gi];
  char* base = p->ws + g.ws_off;
  char* end = base + (size_t)WS_FIELDS * g.bsub * g.n3 * p->es;
  for (int r0 = 0; r0 < g.count; r0 += g.bsub) {
    Ctx c{p, g, st, 2 * p->es, base, std::min(g.bsub, g.count - r0), end};
    const int r = g.rfirst + r0;
    CHK(displace_batch(c, t, noise + r, psi1 + r, psi2 + r));
  }
  return LPT2_OK;
}

// all grids; with several grids, each on its own stream between a fork on s
// and a join back into s (the same sequence records as graph branches)
lpt2_status run_displace(lpt2_plan_t p, const std::vector<Tables*>& tabs, const void* const* noise,
                         void* const* psi1, void* const* psi2, hipStream_t s) {
  if (p->grids.size() == 1) return run_grid(p, 0, tabs[0], noise, psi1, psi2, s);
  hipError_t e = hipEventRecord(p->fork, s);
  if (e != hipSuccess) return hip_fail(p, e, "fork");
  lpt2_status st = LPT2_OK;
  for (size_t i = 0; i < p->grids.size(); ++i) {
    Grid& g = p->grids[i];
    e = hipStreamWaitEvent(g.st, p->fork, 0);
    if (e != hipSuccess && st == LPT2_OK) st = hip_fail(p, e, "fork wait");
    if (st == LPT2_OK) st = run_grid(p, (int)i, tabs[i], noise, psi1, psi2, g.st);
    e = hipEventRecord(g.join, g.st);  // joined also after an error, so a capture can end
    if (e == hipSuccess) e = hipStreamWaitEvent(s, g.join, 0);
    if (e != hipSuccess && st == LPT2_OK) st = hip_fail(p, e, "join");
  }
  return st;
}

// every realisation of grid gi at the n_a scale factors: the full chain at
// a[0], then the epoch chain at a[1..]; psi arrays epoch-major (j * nr + r)
lpt2_status run_grid_epochs(lpt2_plan_t p, int gi, int n_a, const double* a, const void* const* noise,
                            void* const* psi1, void* const* psi2, hipStream_t st) {
  Grid& g = p->grids[gi];
  const int nr_all = (int)p->rgrid.size();
  char* base = p->ws + g.ws_off;
  char* end = base + (size_t)WS_FIELDS * g.bsub * g.n3 * p->es;
  for (int r0 = 0; r0 < g.count; r0 += g.bsub) {
    Ctx c{p, g, st, 2 * p->es, base, std::min(g.bsub, g.count - r0), end};
    const int r = g.rfirst + r0;
    for (int j = 0; j < n_a; ++j) {
      Tables* t = nullptr;  // used at once: a later lookup may move the cache
      CHK(get_tables(p, g, a[j], false, st, &t));
      const size_t o = (size_t)j * nr_all + r;
      if (j == 0)
        CHK(displace_batch(c, t, noise + r, psi1 + o, psi2 + o));
      else
        CHK(epoch_batch(c, t, psi1 + o, psi2 + o));
    }
  }
  return LPT2_OK;
}

lpt2_status run_epochs(lpt2_plan_t p, int n_a, const double* a, const void* const* noise, void* const* psi1,
                       void* const* psi2, hipStream_t s) {
  if (p->grids.size() == 1) return run_grid_epochs(p, 0, n_a, a, noise, psi1, psi2, s);
  hipError_t e = hipEventRecord(p->fork, s);
  if (e != hipSuccess) return hip_fail(p, e, "fork");
  lpt2_status st = LPT2_OK;
  for (size_t i = 0; i < p->grids.size(); ++i) {
    Grid& g = p->grids[i];
    e = hipStreamWaitEvent(g.st, p->fork, 0);
    if (e != hipSuccess && st == LPT2_OK) st = hip_fail(p, e, "fork wait");
    if (st == LPT2_OK) st = run_grid_epochs(p, (int)i, n_a, a, noise, psi1, psi2, g.st);
    e = hipEventRecord(g.join, g.st);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, g.join, 0);
    if (e != hipSuccess && st == LPT2_OK) st = hip_fail(p, e, "join");
  }
  return st;
}

// the captured graph of the whole batch for (a, these buffers)
lpt2_status graph_for(lpt2_plan_t p, double a, const std::vector<Tables*>& tabs, const void* const* noise,
                      void* const* psi1, void* const* psi2, GraphEntry** out) {
  const size_t nr = p->rgrid.size();
  std::vector<const void*> key(3 * nr);
  for (size_t r = 0; r < nr; ++r) {
    key[3 * r] = noise[r];
    key[3 * r + 1] = psi1[r];
    key[3 * r + 2] = psi2[r];
  }
  for (auto& ge : p->graphs)
    if (ge.a == a && ge.ptrs == key) {
      *out = &ge;
      return LPT2_OK;
    }
  if (p->graphs.size() >= 8) {  // keep a few; the oldest may still run
    (void)hipDeviceSynchronize();
    (void)hipGraphExecDestroy(p->graphs.front().exec);
    (void)hipGraphDestroy(p->graphs.front().graph);
    p->graphs.erase(p->graphs.begin());
  }
  hipStream_t cs = p->cap_stream;
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) return hip_fail(p, e, "begin capture");
  p->capturing = true;
  lpt2_status st = run_displace(p, tabs, noise, psi1, psi2, cs);
  p->capturing = false;
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(cs, &graph);
  if (st != LPT2_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return hip_fail(p, e, "end capture");
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return hip_fail(p, e, "graph instantiate");
  }
  p->graphs.push_back({a, key, graph, exec});
  *out = &p->graphs.back();
  return LPT2_OK;
}

lpt2_status set_tiles(lpt2_plan_t p, Grid& g, const int* tiles) {
  for (int k = 0; k < 3; ++k) {
    bool ok = tiles[k] == 0;
    for (int i = 0; i < 3; ++i) ok = ok || tiles[k] == col_width(p->prec, g.n, k, i);
    if (!ok) return fail(p, LPT2_EINVAL, "tile width " + std::to_string(tiles[k]) + " not offered for this grid");
  }
  bool same = true;
  for (int k = 0; k < 3; ++k) same = same && g.tiles[k] == tiles[k];
  if (same) return LPT2_OK;
  (void)hipDeviceSynchronize();
  drop_graphs(p);  // graphs hold the old launch shapes
  for (int k = 0; k < 3; ++k) g.tiles[k] = tiles[k];
  return LPT2_OK;
}

// ---- tile tuner ------------------------------------------------------------------
// Times every combination of the offered tile widths (single y/x passes,
// fused y pass, fused x pass) on the grid's own batch and keeps the fastest.
// Results are cached in a text file, one line per (device, precision, n,
// batch):  lpt2-tiles <arch> <fp32|fp64> <n> <batch> <col> <y> <x>
std::string tune_key(lpt2_plan_t p, const Grid& g) {
  int dev = 0;
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);
  }
  return arch + " " + (p->prec == PREC_F32 ? "fp32" : "fp64") + " " + std::to_string(g.n) + " " +
         std::to_string(g.bsub);
}

bool tune_lookup(const char* path, const std::string& key, int* tiles) {
  if (!path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  while (std::fgets(line, sizeof(line), f)) {
    char arch[128], prec[16];
    int n = 0, b = 0, t0 = 0, t1 = 0, t2 = 0;
    if (std::sscanf(line, "lpt2-tiles %127s %15s %d %d %d %d %d", arch, prec, &n, &b, &t0, &t1, &t2) != 7) continue;
    const std::string k = std::string(arch) + " " + prec + " " + std::to_string(n) + " " + std::to_string(b);
    if (k == key) {  // the last matching line wins
      tiles[0] = t0;
      tiles[1] = t1;
      tiles[2] = t2;
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

// minimum over `reps` timed runs of grid gi (after one warm run)
lpt2_status time_grid(lpt2_plan_t p, int gi, const Tables* t, const void* const* noise, void* const* psi1,
                      void* const* psi2, hipStream_t s, int reps, float* best) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return hip_fail(p, e, "tuner events");
  }
  lpt2_status st = run_grid(p, gi, t, noise, psi1, psi2, s);
  *best = 1e30f;
  for (int i = 0; i < reps && st == LPT2_OK; ++i) {
    (void)hipEventRecord(e0, s);
    st = run_grid(p, gi, t, noise, psi1, psi2, s);
    (void)hipEventRecord(e1, s);
    float ms = 0.f;
    if (st == LPT2_OK && hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
      *best = std::min(*best, ms);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

lpt2_status autotune(lpt2_plan_t p, const std::vector<Tables*>& tabs, const void* const* noise, void* const* psi1,
                     void* const* psi2, const char* path, hipStream_t s) {
  const bool prof = p->prof;
  p->prof = false;
  lpt2_status st = LPT2_OK;
  std::string lines;
  for (size_t gi = 0; gi < p->grids.size() && st == LPT2_OK; ++gi) {
    Grid& g = p->grids[gi];
    const std::string key = tune_key(p, g);
    int tiles[3];
    if (tune_lookup(path, key, tiles) && set_tiles(p, g, tiles) == LPT2_OK) continue;
    int opt[3][3], nopt[3] = {0, 0, 0};  // distinct widths per pass kind
    for (int k = 0; k < 3; ++k)
      for (int i = 0; i < 3; ++i) {
        const int w = col_width(p->prec, g.n, k, i);
        bool dup = false;
        for (int j = 0; j < nopt[k]; ++j) dup = dup || opt[k][j] == w;
        if (!dup) opt[k][nopt[k]++] = w;
      }
    float best = 1e30f;
    int bt[3] = {0, 0, 0};
    for (int i0 = 0; i0 < nopt[0] && st == LPT2_OK; ++i0)
      for (int i1 = 0; i1 < nopt[1] && st == LPT2_OK; ++i1)
        for (int i2 = 0; i2 < nopt[2] && st == LPT2_OK; ++i2) {
          const int tt[3] = {opt[0][i0], opt[1][i1], opt[2][i2]};
          st = set_tiles(p, g, tt);
          float ms = 0.f;
          if (st == LPT2_OK) st = time_grid(p, (int)gi, tabs[gi], noise, psi1, psi2, s, 3, &ms);
          if (st == LPT2_OK && ms < best) {
            best = ms;
            std::memcpy(bt, tt, sizeof(bt));
          }
        }
    if (st == LPT2_OK) st = set_tiles(p, g, bt);
    if (st == LPT2_OK)
      lines += "lpt2-tiles " + key + " " + std::to_string(bt[0]) + " " + std::to_string(bt[1]) + " " +
               std::to_string(bt[2]) + "\n";
  }
  p->prof = prof;
  if (st == LPT2_OK && path && !lines.empty()) {
    FILE* f = std::fopen(path, "a");
    if (!f) return fail(p, LPT2_EINVAL, std::string("cannot append to tuning cache ") + path);
    std::fputs(lines.c_str(), f);
    std::fclose(f);
  }
  return st;
}

// bodies of lpt2_source_spectrum and lpt2_triangle_ratio (the caller holds the plan)
lpt2_status spectrum_impl(lpt2_plan_t p, Grid& g, double a, const void* noise, int nbins, int quantity,
                                 double* k_mean, double* count, double* mean, double* std_dev, hipStream_t s) {
  Tables* t = nullptr;
  CHK(get_tables(p, g, a, false, s, &t));
  Ctx c{p, g, s, 2 * p->es, p->ws, 1};
  const double kf = 2.0 * kPi / g.cfg.box;
  if (quantity == LPT2_SPEC_POWER) {
    CHK(source_k(c, t, noise, 11, 1.0));
    const double n3 = (double)g.n3;
    const double qs = g.cfg.box * g.cfg.box * g.cfg.box / (n3 * n3);
    RUN("shell_bin", 0.0,
        launch_bin(p->prec, g.n, c.slot(11), c.cap(c.slot(11)), nullptr, 0, 0, qs, nbins, kf, p->bin_partial,
                   p->bin_out, s));
  } else {
    Tables* tg = nullptr;
    CHK(get_tables(p, g, a, true, s, &tg));
    double d1gr = 0.0;
    hipError_t e = hipMemcpyAsync(&d1gr, tg->d1n, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(p, e, "D1_GR readback");
    const double G = four_pi_g_rho(g.c, a);
    CHK(source_k(c, t, noise, 11, -G * d1gr * d1gr));
    CHK(mg_source_k(c, t, noise));
    RUN("shell_bin", 0.0,
        launch_bin(p->prec, g.n, c.slot(10), c.cap(c.slot(10)), c.slot(11), c.cap(c.slot(11)), 1, 1.0, nbins, kf,
                   p->bin_partial, p->bin_out, s));
  }
  std::vector<double> h(4 * (size_t)nbins);
  hipError_t e = hipMemcpyAsync(h.data(), p->bin_out, sizeof(double) * 4 * nbins, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(p, e, "spectrum readback");
  for (int i = 0; i < nbins; ++i) {
    k_mean[i] = h[i];
    count[i] = h[nbins + i];
    mean[i] = h[2 * nbins + i];
    std_dev[i] = h[3 * nbins + i];
  }
  return LPT2_OK;
}

lpt2_status triangle_impl(lpt2_plan_t p, Grid& g, double a, double ratio, double theta_deg, int winther,
                                 const double* k, int nk, double* out) {
  hipStream_t s = nullptr;
  Tables *t = nullptr, *tg = nullptr;
  CHK(get_tables(p, g, a, false, s, &t));
  CHK(get_tables(p, g, a, true, s, &tg));
  const int n = g.cfg.nk_growth;
  std::vector<double> d1(n), d1g(1);
  hipError_t e = hipMemcpy(d1.data(), t->d1n, sizeof(double) * n, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(d1g.data(), tg->d1n, sizeof(double), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(p, e, "growth readback");
  const double cs = cos_deg(theta_deg);
  for (int i = 0; i < nk; ++i) {
    double k1, k2;
    triangle(k[i], ratio, cs, k1, k2);
    const double dd = winther ? std::pow(interp_lnk(d1.data(), n, g.lkmin, g.lkmax, k[i]), 2)
                              : interp_lnk(d1.data(), n, g.lkmin, g.lkmax, k1) * interp_lnk(d1.data(), n, g.lkmin, g.lkmax, k2);
    out[i] = dd * brace(g.c, k[i], k1, k2, cs, a) / (d1g[0] * d1g[0] * (1.0 - cs * cs));
  }
  return LPT2_OK;
}

// The fit of the factorisation choice: the cheapest candidate for grid g at a
// (count-weighted squared misfit of the binned ratio, shells 0 < k <= kcut).
lpt2_status fit_candidates(lpt2_plan_t p, Grid& g, double a, const void* noise, int nbins, double kcut,
                                  hipStream_t s, int* best, double* costs) {
  std::vector<double> km(nbins), cnt(nbins), mean(nbins), sd(nbins);
  CHK(spectrum_impl(p, g, a, noise, nbins, LPT2_SPEC_RATIO, km.data(), cnt.data(), mean.data(), sd.data(), s));
  std::vector<double> ks, ws, ms;
  for (int i = 0; i < nbins; ++i)
    if (cnt[i] > 0.0 && km[i] > 0.0 && km[i] <= kcut) {
      ks.push_back(km[i]);
      ws.push_back(cnt[i]);
      ms.push_back(mean[i]);
    }
  if (ks.empty()) return fail(p, LPT2_EINVAL, "no populated shell with 0 < k <= kcut");
  std::vector<double> rt(ks.size());
  int bi = -1;
  double bc = 0.0;
  for (int c = 0; c < kNCandidates; ++c) {
    const Candidate& q = kCandidates[c];
    CHK(triangle_impl(p, g, a, q.ratio, q.theta, q.winther, ks.data(), (int)ks.size(), rt.data()));
    double cost = 0.0;
    for (size_t i = 0; i < ks.size(); ++i) cost += ws[i] * (ms[i] - rt[i]) * (ms[i] - rt[i]);
    if (costs) costs[c] = cost;
    if (bi < 0 || cost < bc) {
      bi = c;
      bc = cost;
    }
  }
  *best = bi;
  return LPT2_OK;
}

void set_auto(Grid& g, double a, int cand) {
  for (auto& c : g.auto_choice)
    if (c.first == a) {
      c.second = cand;
      return;
    }
  g.auto_choice.push_back({a, cand});
}

// AUTO configurations: the factorisation at a is chosen once, from the
// source ratio of `noise` (n/2 shells of width k_f, k <= 0.4 h/Mpc).
lpt2_status resolve_auto(lpt2_plan_t p, Grid& g, double a, const void* noise, hipStream_t s) {
  if (g.cfg.factorisation != LPT2_D2_AUTO || auto_lookup(g, a) != kAutoNone) return LPT2_OK;
  int best = 0;
  CHK(fit_candidates(p, g, a, noise, std::min(g.n / 2, BIN_MAXBINS), 0.4, s, &best, nullptr));
  set_auto(g, a, best);
  return LPT2_OK;
}

}  // namespace

// =============================================================================
// C ABI
// =============================================================================
extern "C" {

void lpt2_config_default(lpt2_config* c) {
  if (!c) return;
  std::memset(c, 0, sizeof(*c));
  c->n = 32;
  c->box = 128.0;
  c->omega_m = 0.3;
  c->h = 0.7;
  c->n_s = 0.96;
  c->sigma8 = 0.8;
  c->gravity = LPT2_GRAV_GR;
  c->fr0_abs = 1e-5;
  c->hs_n = 1;
  c->mu_const = 1.0;
  c->factorisation = LPT2_D2_EDS;
  c->tri_ratio = 1.0;
  c->tri_theta_deg = 90.0;
  c->nk_growth = 256;
  c->kmin = 1e-3;
  c->kmax = 10.0;
  c->a_init = 1e-3;
  c->ode_steps = 4096;
  c->precision = LPT2_FP64;
}

const char* lpt2_strerror(lpt2_status s) {
  // read as an int: callers through C or ctypes may pass any int, and a value
  // outside the enumerators must not be loaded as an lpt2_status
  int v = 0;
  std::memcpy(&v, &s, sizeof(v));
  switch (v) {
    case LPT2_OK: return "ok";
    case LPT2_EINVAL: return "invalid argument";
    case LPT2_EUNSUPPORTED: return "unsupported";
    case LPT2_ENOMEM: return "out of memory";
    case LPT2_EDEVICE: return "device error";
    case LPT2_ESTATE: return "plan busy or in the wrong state";
  }
  return "unknown status";
}

const char* lpt2_last_error(lpt2_plan_t p) { return p ? p->err.c_str() : g_err.c_str(); }

lpt2_status lpt2_plan(const lpt2_config* cfgs, int n_cfgs, const int* counts, lpt2_plan_t* out) {
  g_alloc_count = 0;
  if (!out) return fail(nullptr, LPT2_EINVAL, "out is NULL");
  *out = nullptr;
  if (!cfgs || n_cfgs < 1) return fail(nullptr, LPT2_EINVAL, "need at least one configuration");
  int prec = cfgs[0].precision;
  for (int i = 0; i < n_cfgs; ++i) {
    std::string why;
    lpt2_status st = validate(cfgs[i], why);
    if (st != LPT2_OK) return fail(nullptr, st, "config " + std::to_string(i) + ": " + why);
    if (cfgs[i].precision != prec) return fail(nullptr, LPT2_EUNSUPPORTED, "all configurations must share a precision");
    if (counts && counts[i] < 1) return fail(nullptr, LPT2_EINVAL, "counts must be >= 1");
  }
  lpt2_plan_s* p = new lpt2_plan_s();
  p->prec = prec == LPT2_FP32 ? PREC_F32 : PREC_F64;
  p->es = p->prec == PREC_F32 ? 4 : 8;
  size_t maxf = 0;
  for (int i = 0; i < n_cfgs; ++i) {
    Grid g;
    g.cfg = cfgs[i];
    g.count = counts ? counts[i] : 1;
    g.n = cfgs[i].n;
    g.m = g.n / 2;
    g.nnm = (long)g.n * g.n * g.m;
    g.n3 = (long)g.n * g.n * g.n;
    g.n2cnt = 3L * g.m * g.m + 1;
    g.c.om = cfgs[i].omega_m;
    g.c.ol = 1.0 - cfgs[i].omega_m;
    g.c.h = cfgs[i].h;
    g.c.ns = cfgs[i].n_s;
    g.c.gravity = cfgs[i].gravity == LPT2_GRAV_FR_HS ? GRAV_FR : (cfgs[i].gravity == LPT2_GRAV_MU_CONST ? GRAV_MUC : GRAV_GR);
    g.c.fr0 = cfgs[i].fr0_abs;
    g.c.mu0 = cfgs[i].mu_const;
    g.amp = sigma8_amplitude(g.c, cfgs[i].sigma8);
    g.lkmin = std::log(cfgs[i].kmin);
    g.lkmax = std::log(cfgs[i].kmax);
    // twiddles exp(-2 pi i m / n), m < n, from long double, rounded once
    std::vector<double> tw64(2 * g.n);
    std::vector<float> tw32(2 * g.n);
    for (int m = 0; m < g.n; ++m) {
      const long double ang = -2.0L * 3.14159265358979323846264338327950288L * (long double)m / (long double)g.n;
      tw64[2 * m] = (double)cosl(ang);
      tw64[2 * m + 1] = (double)sinl(ang);
      tw32[2 * m] = (float)cosl(ang);
      tw32[2 * m + 1] = (float)sinl(ang);
    }
    const size_t twb = (size_t)2 * g.n * p->es;
    hipError_t e = dev_malloc(&g.tw, twb);
    if (e != hipSuccess) {
      p->grids.push_back(g);
      lpt2_destroy(p);
      return fail(nullptr, LPT2_ENOMEM, "twiddle allocation failed");
    }
    e = hipMemcpy(g.tw, p->prec == PREC_F32 ? (const void*)tw32.data() : (const void*)tw64.data(), twb,
                  hipMemcpyHostToDevice);
    p->grids.push_back(g);
    if (e != hipSuccess) {
      lpt2_destroy(p);
      return fail(nullptr, LPT2_EDEVICE, std::string("twiddle upload: ") + hipGetErrorString(e));
    }
    for (int r = 0; r < p->grids.back().count; ++r) p->rgrid.push_back(i);
    const size_t fbytes = (size_t)g.n3 * p->es;
    if (fbytes > maxf) maxf = fbytes;
  }
  // batches: each grid gets a region of WS_FIELDS slots of bsub realisations
  // (bsub as large as the batch budget and the per-launch pointer table allow)
  size_t region_total = 0;
  int rfirst = 0;
  for (auto& g : p->grids) {
    const size_t per = (size_t)WS_FIELDS * g.n3 * p->es;
    size_t b = BATCH_WS_BUDGET / per;
    if (b < 1) b = 1;
    if (b > (size_t)BATCH_MAX) b = BATCH_MAX;
    if (b > (size_t)g.count) b = g.count;
    g.bsub = (int)b;
    g.rfirst = rfirst;
    rfirst += g.count;
    g.ws_off = region_total;
    region_total += per * b;
  }
  p->ws_bytes = std::max(maxf * WS_FIELDS, region_total);
  hipError_t e = dev_malloc((void**)&p->ws, p->ws_bytes);
  if (e != hipSuccess) {
    p->ws = nullptr;
    lpt2_destroy(p);
    return fail(nullptr, LPT2_ENOMEM, "workspace allocation failed");
  }
  if (p->grids.size() > 1) {  // grids of a plan run side by side on streams of their own
    e = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming);
    for (auto& g : p->grids) {
      if (e == hipSuccess) e = hipStreamCreateWithFlags(&g.st, hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&g.join, hipEventDisableTiming);
    }
    if (e != hipSuccess) {
      lpt2_destroy(p);
      return fail(nullptr, LPT2_EDEVICE, std::string("stream setup: ") + hipGetErrorString(e));
    }
  }
  // the binner's partial sums and bins, the lpt2_check_finite counter, and
  // each grid's 16 tile-ticket words (64 bytes, zeroed here once: the
  // kernels leave them at zero)
  const size_t small_bytes = sizeof(double) * (BIN_BLOCKS * (size_t)BIN_MAXBINS * 4 + 4 * BIN_MAXBINS) + 256;
  e = dev_malloc((void**)&p->bin_partial, small_bytes + 64 * p->grids.size());
  if (e != hipSuccess) {
    p->bin_partial = nullptr;
    lpt2_destroy(p);
    return fail(nullptr, LPT2_ENOMEM, "binner allocation failed");
  }
  e = hipMemset(reinterpret_cast<char*>(p->bin_partial) + small_bytes, 0, 64 * p->grids.size());
  if (e != hipSuccess) {
    lpt2_destroy(p);
    return fail(nullptr, LPT2_EDEVICE, std::string("tile tickets: ") + hipGetErrorString(e));
  }
  p->bin_out = p->bin_partial + (size_t)BIN_BLOCKS * BIN_MAXBINS * 4;
  p->counter = reinterpret_cast<unsigned long long*>(p->bin_out + 4 * BIN_MAXBINS);
  for (size_t i = 0; i < p->grids.size(); ++i)
    p->grids[i].tq = reinterpret_cast<unsigned*>(reinterpret_cast<char*>(p->bin_partial) + small_bytes + 64 * i);
  char* scr = nullptr;  // the allocation-free entry point's memory on this device
  lpt2_status sst = scratch_address(p, &scr);
  if (sst != LPT2_OK) {
    const std::string msg = p->err;
    lpt2_destroy(p);
    return fail(nullptr, sst, msg);
  }
  *out = p;
  return LPT2_OK;
}

lpt2_status lpt2_destroy(lpt2_plan_t p) {
  if (!p) return LPT2_OK;
  (void)hipDeviceSynchronize();
  drop_graphs(p);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  if (p->fork) (void)hipEventDestroy(p->fork);
  for (auto& g : p->grids) {
    if (g.st) (void)hipStreamDestroy(g.st);
    if (g.join) (void)hipEventDestroy(g.join);
    if (g.tw) (void)hipFree(g.tw);
    for (auto& t : g.tables) {
      (void)hipFree(t.d1n);
      if (t.radial) (void)hipFree(t.radial);
    }
    for (auto& t : g.gr_tables) (void)hipFree(t.d1n);
  }
  if (p->ws) (void)hipFree(p->ws);
  if (p->bin_partial) (void)hipFree(p->bin_partial);
  prof_flush(p);
  for (auto e : p->pool) (void)hipEventDestroy(e);
  delete p;
  return LPT2_OK;
}

int lpt2_realisations(lpt2_plan_t p) { return p ? (int)p->rgrid.size() : 0; }

lpt2_status lpt2_realisation_info(lpt2_plan_t p, int r, int* n, int* precision) {
  if (!p) return fail(nullptr, LPT2_EINVAL, "plan is NULL");
  if (r < 0 || r >= (int)p->rgrid.size()) return fail(p, LPT2_EINVAL, "realisation index out of range");
  if (n) *n = p->grids[p->rgrid[r]].n;
  if (precision) *precision = p->prec == PREC_F32 ? LPT2_FP32 : LPT2_FP64;
  return LPT2_OK;
}

long long lpt2_workspace_bytes(lpt2_plan_t p) { return p ? (long long)p->ws_bytes : 0; }

lpt2_status lpt2_displace(lpt2_plan_t p, double a, const void* const* noise, void* const* psi1, void* const* psi2,
                          void* stream) {
  if (!p) return fail(nullptr, LPT2_EINVAL, "plan is NULL");
  Busy b(p);
  if (!b.ok) return fail(p, LPT2_ESTATE, "plan is in use by another call");
  CHK(check_a(p, a));
  if (!noise || !psi1 || !psi2) return fail(p, LPT2_EINVAL, "null pointer array");
  const int nr = (int)p->rgrid.size();
  for (int r = 0; r < nr; ++r)
    if (!noise[r] || !psi1[r] || !psi2[r]) return fail(p, LPT2_EINVAL, "null field pointer for realisation " + std::to_string(r));
  hipStream_t s = (hipStream_t)stream;
  for (auto& g : p->grids) CHK(resolve_auto(p, g, a, noise[g.rfirst], s));  // before any capture
  std::vector<Tables*> tabs;
  CHK(tables_for(p, a, s, tabs));
  if (!p->graph_mode) return run_displace(p, tabs, noise, psi1, psi2, s);
  GraphEntry* ge = nullptr;
  CHK(graph_for(p, a, tabs, noise, psi1, psi2, &ge));
  hipError_t e = hipGraphLaunch(ge->exec, s);
  if (e != hipSuccess) return hip_fail(p, e, "graph launch");
  return LPT2_OK;
}

lpt2_status lpt2_displace_noalloc(lpt2_plan_t p, double a, const void* noise, void* psi1, void* psi2,
                                  void* stream) {
  if (!p) return fail(nullptr, LPT2_EINVAL, "plan is NULL");
  Busy b(p);
  if (!b.ok) return fail(p, LPT2_ESTATE, "plan is in use by another call");
  CHK(check_a(p, a));
  if (!noise || !psi1 || !psi2) return fail(p, LPT2_EINVAL, "null pointer");
  if (p->rgrid.size() != 1) return fail(p, LPT2_EUNSUPPORTED, "lpt2_displace_noalloc takes plans of one realisation");
  Grid& g = p->grids[0];
  const size_t slots = (size_t)WS_FIELDS * g.n3 * p->es;
  if (slots > kScratchSlotBytes)
    return fail(p, LPT2_EUNSUPPORTED, "grid of " + std::to_string(g.n) + "^3 needs " + std::to_string(slots) +
                                          " bytes of scratch; the static scratch holds " +
                                          std::to_string(kScratchSlotBytes) + " (FP32 n <= 96, FP64 n <= 64)");
  const size_t tabs = sizeof(double) * (2 * (size_t)g.cfg.nk_growth + (size_t)TAB_ROWS * g.n2cnt) + 256;
  if (tabs > kScratchTableBytes) return fail(p, LPT2_EUNSUPPORTED, "growth tables do not fit the static scratch");
  if (g.cfg.factorisation == LPT2_D2_AUTO && auto_lookup(g, a) == kAutoNone)
    return fail(p, LPT2_ESTATE, "AUTO factorisation not chosen at this a (run lpt2_displace or "
                                "lpt2_choose_factorisation first)");
  char* base = nullptr;
  CHK(scratch_address(p, &base));
  hipStream_t s = (hipStream_t)stream;
  struct Quiet {  // no per-launch profiling events (creating one may allocate)
    lpt2_plan_t p;
    explicit Quiet(lpt2_plan_t q) : p(q) { p->quiet = true; }
    ~Quiet() { p->quiet = false; }
  } quiet(p);
  // the plan's tables at a if it has them, else built into the scratch (not kept)
  Tables local;
  const Tables* t = find_tables(g, a, false);
  if (!t) {
    char* tb = base + kScratchSlotBytes;
    local.d1n = (double*)tb;
    local.d2n = local.d1n + g.cfg.nk_growth;
    local.radial = (double*)(tb + ((sizeof(double) * 2 * (size_t)g.cfg.nk_growth + 255) & ~(size_t)255));
    CHK(build_tables_into(p, g, a, false, false, s, local));
    t = &local;
  }
  Ctx c{p, g, s, 2 * p->es, base, 1, base + kScratchSlotBytes, base};
  const void* in[1] = {noise};
  void* o1[1] = {psi1};
  void* o2[1] = {psi2};
  return displace_batch(c, t, in, o1, o2);
}

lpt2_status lpt2_displace_epochs(lpt2_plan_t p, int n_a, const double* a, const void* const* noise,
                                 void* const* psi1, void* const* psi2, void* stream) {
  if (!p) return fail(nullptr, LPT2_EINVAL, "plan is NULL");
  Busy b(p);
  if (!b.ok) return fail(p, LPT2_ESTATE, "plan is in use by another call");
  if (n_a < 1 || n_a > LPT2_MAX_EPOCHS || !a) return fail(p, LPT2_EINVAL, "need 1..16 scale factors");
  for (int j = 0; j < n_a; ++j) CHK(check_a(p, a[j]));
  if (!noise || !psi1 || !psi2) return fail(p, LPT2_EINVAL, "null pointer array");
  const int nr = (int)p->rgrid.size();
  for (int r = 0; r < nr; ++r)
    if (!noise[r]) return fail(p, LPT2_EINVAL, "null noise pointer for realisation " + std::to_string(r));
  for (int i = 0; i < n_a * nr; ++i)
    if (!psi1[i] || !psi2[i]) return fail(p, LPT2_EINVAL, "null output pointer at " + std::to_string(i));
  hipStream_t s = (hipStream_t)stream;
  for (int j = 0; j < n_a; ++j)
    for (auto& g : p->grids) CHK(resolve_auto(p, g, a[j], noise[g.rfirst], s));
  return run_epochs(p, n_a, a, noise, psi1, psi2, s);
}

lpt2_status lpt2_set_graph(lpt2_plan_t p, int enable) {
  if (!p) return fail(nullptr, LPT2_EINVAL, "plan is NULL");
  Busy b(p);
  if (!b.ok) return fail(p, LPT2_ESTATE, "plan is in use by another call");
  if (enable && !p->cap_stream) {
    hipError_t e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      p->cap_stream = nullptr;
      return hip_fail(p, e, "capture stream");
    }
  }
  if (!enable) {
    (void)hipDeviceSynchronize();
    drop_graphs(p);
  }
  p->graph_mode = enable != 0;
  return LPT2_OK;
}

lpt2_status lpt2_get_tiles(lpt2_plan_t p, int grid, int* tiles) {
  if (!p) return fail(nullptr, LPT2_EINVAL, "plan is NULL");
  if (!tiles || grid < 0 || grid >= (int)p->grids.size()) return fail(p, LPT2_EINVAL, "bad grid index or NULL");
  const Grid& g = p->grids[grid];
  for (int k = 0; k < 3; ++k) tiles[k] = g.tiles[k] ? g.tiles[k] : default_width(p->prec, g.n, k);
  return LPT2_OK;
}

lpt2_status lpt2_tile_options(lpt2_plan_t p, int grid, int* widths) {
  if (!p) return fail(nullptr, LPT2_EINVAL, "plan is NULL");
  if (!widths || grid < 0 || grid >= (int)p->grids.size()) return fail(p, LPT2_EINVAL, "bad grid index or NULL");
  for (int k = 0; k < 3; ++k)
    for (int i = 0; i < 3; ++i) widths[3 * k + i] = col_width(p->prec, p->grids[grid].n, k, i);
  return LPT2_OK;
}

lpt2_status lpt2_set_tiles(lpt2_plan_t p, int grid, const int* tiles) {
  if (!p) return fail(nullptr, LPT2_EINVAL, "plan is NULL");
  Busy b(p);
  if (!b.ok) return fail(p, LPT2_ESTATE, "plan is in use by another call");
  if (!tiles || grid < 0 || grid >= (int)p->grids.size()) return fail(p, LPT2_EINVAL, "bad grid index or NULL");
  CHK(set_tiles(p, p->grids[grid], tiles));
  return LPT2_OK;
}

lpt2_status lpt2_autotune(lpt2_plan_t p, double a, const void* const* noise, void* const* psi1, void* const* psi2,
                          const char* cache_path, void* stream) {
  if (!p) return fail(nullptr, LPT2_EINVAL, "plan is NULL");
  Busy b(p);
  if (!b.ok) return fail(p, LPT2_ESTATE, "plan is in use by another call");
  CHK(check_a(p, a));
  if (!noise || !psi1 || !psi2) return fail(p, LPT2_EINVAL, "null pointer array");
  const int nr = (int)p->rgrid.size();
  for (int r = 0; r < nr; ++r)
    if (!noise[r] || !psi1[r] || !psi2[r]) return fail(p, LPT2_EINVAL, "null field pointer for realisation " + std::to_string(r));
  hipStream_t s = (hipStream_t)stream;
  for (auto& g : p->grids) CHK(resolve_auto(p, g, a, noise[g.rfirst], s));
  std::vector<Tables*> tabs;
  CHK(tables_for(p, a, s, tabs));
  return autotune(p, tabs, noise, psi1, psi2, cache_path, s);
}

lpt2_status lpt2_source_spectrum(lpt2_plan_t p, double a, const void* noise, int nbins, int quantity, double* k_mean,
                                 double* count, double* mean, double* std_dev, void* stream) {
  if (!p) return fail(nullptr, LPT2_EINVAL, "plan is NULL");
  Busy b(p);
  if (!b.ok) return fail(p, LPT2_ESTATE, "plan is in use by another call");
  CHK(check_a(p, a));
  if (!noise || !k_mean || !count || !mean || !std_dev) return fail(p, LPT2_EINVAL, "null pointer");
  if (nbins < 1 || nbins > BIN_MAXBINS) return fail(p, LPT2_EINVAL, "nbins must be in 1..512");
  if (quantity != LPT2_SPEC_POWER && quantity != LPT2_SPEC_RATIO) return fail(p, LPT2_EINVAL, "unknown quantity");
  hipStream_t s = (hipStream_t)stream;
  Grid& g = p->grids[p->rgrid[0]];
  CHK(resolve_auto(p, g, a, noise, s));
  return spectrum_impl(p, g, a, noise, nbins, quantity, k_mean, count, mean, std_dev, s);
}

lpt2_status lpt2_triangle_ratio(lpt2_plan_t p, double a, double ratio, double theta_deg, int winther, const double* k,
                                int nk, double* out) {
  if (!p) return fail(nullptr, LPT2_EINVAL, "plan is NULL");
  Busy b(p);
  if (!b.ok) return fail(p, LPT2_ESTATE, "plan is in use by another call");
  CHK(check_a(p, a));
  if (!k || !out || nk < 0) return fail(p, LPT2_EINVAL, "null pointer");
  if (!(ratio > 0.0) || !(theta_deg > 0.0 && theta_deg < 180.0)) return fail(p, LPT2_EINVAL, "bad triangle");
  return triangle_impl(p, p->grids[p->rgrid[0]], a, ratio, theta_deg, winther, k, nk, out);
}

int lpt2_factorisation_candidates(void) { return kNCandidates; }

lpt2_status lpt2_factorisation_candidate(int i, const char** name, double* ratio, double* theta_deg, int* winther) {
  if (i < 0 || i >= kNCandidates) return fail(nullptr, LPT2_EINVAL, "candidate index out of range");
  if (name) *name = kCandidates[i].name;
  if (ratio) *ratio = kCandidates[i].ratio;
  if (theta_deg) *theta_deg = kCandidates[i].theta;
  if (winther) *winther = kCandidates[i].winther;
  return LPT2_OK;
}

lpt2_status lpt2_choose_factorisation(lpt2_plan_t p, double a, const void* noise, int nbins, double kcut, int apply,
                                      int* best, double* costs, void* stream) {
  if (!p) return fail(nullptr, LPT2_EINVAL, "plan is NULL");
  Busy b(p);
  if (!b.ok) return fail(p, LPT2_ESTATE, "plan is in use by another call");
  CHK(check_a(p, a));
  if (!noise || !best) return fail(p, LPT2_EINVAL, "null pointer");
  if (nbins < 1 || nbins > BIN_MAXBINS) return fail(p, LPT2_EINVAL, "nbins must be in 1..512");
  if (!(kcut > 0.0)) return fail(p, LPT2_EINVAL, "kcut must be > 0");
  Grid& g = p->grids[p->rgrid[0]];
  int bi = 0;
  CHK(fit_candidates(p, g, a, noise, nbins, kcut, (hipStream_t)stream, &bi, costs));
  *best = bi;
  if (!apply) return LPT2_OK;
  if (g.cfg.factorisation == LPT2_D2_AUTO) {  // the tables at a are rebuilt on their next use
    set_auto(g, a, bi);
    return LPT2_OK;
  }
  // a fixed factorisation is replaced by the chosen candidate at every a
  const Candidate& q = kCandidates[bi];
  (void)hipDeviceSynchronize();
  drop_graphs(p);
  if (q.winther) {
    g.cfg.factorisation = LPT2_D2_WINTHER;
  } else if (q.ratio == 1.0 && q.theta == 90.0) {
    g.cfg.factorisation = LPT2_D2_T1;
  } else {
    g.cfg.factorisation = LPT2_D2_TRIANGLE;
    g.cfg.tri_ratio = q.ratio;
    g.cfg.tri_theta_deg = q.theta;
  }
  for (auto& t : g.tables) free_tables(t);  // D2 changes; rebuilt on the next call
  g.tables.clear();
  return LPT2_OK;
}

lpt2_status lpt2_auto_choice(lpt2_plan_t p, int grid, double a, int* candidate) {
  if (!p) return fail(nullptr, LPT2_EINVAL, "plan is NULL");
  if (!candidate || grid < 0 || grid >= (int)p->grids.size()) return fail(p, LPT2_EINVAL, "bad grid index or NULL");
  *candidate = auto_lookup(p->grids[grid], a);
  return LPT2_OK;
}

lpt2_status lpt2_displace_delta(lpt2_plan_t p, double a, const void* delta, void* psi1, void* psi2, void* stream) {
  if (!p) return fail(nullptr, LPT2_EINVAL, "plan is NULL");
  Busy b(p);
  if (!b.ok) return fail(p, LPT2_ESTATE, "plan is in use by another call");
  CHK(check_a(p, a));
  if (!delta || !psi1 || !psi2) return fail(p, LPT2_EINVAL, "null pointer");
  Grid& g = p->grids[p->rgrid[0]];
  if (g.cfg.factorisation == LPT2_D2_AUTO && auto_lookup(g, a) == kAutoNone)
    return fail(p, LPT2_ESTATE, "AUTO factorisation not chosen at this a (run lpt2_displace or "
                                "lpt2_choose_factorisation first)");
  hipStream_t s = (hipStream_t)stream;
  Tables* t = nullptr;
  CHK(get_tables(p, g, a, false, s, &t, true));
  Ctx c{p, g, s, 2 * p->es, p->ws, 1};
  const void* in[1] = {delta};
  void* o1[1] = {psi1};
  void* o2[1] = {psi2};
  return displace_batch(c, t, in, o1, o2);
}

lpt2_status lpt2_matter_power(lpt2_plan_t p, const void* psi1, const void* psi2, int nbins, int flags,
                              double* k_mean, double* count, double* mean, double* std_dev, void* stream) {
  if (!p) return fail(nullptr, LPT2_EINVAL, "plan is NULL");
  Busy b(p);
  if (!b.ok) return fail(p, LPT2_ESTATE, "plan is in use by another call");
  if (!psi1 || !psi2 || !k_mean || !count || !mean || !std_dev) return fail(p, LPT2_EINVAL, "null pointer");
  if (nbins < 1 || nbins > BIN_MAXBINS) return fail(p, LPT2_EINVAL, "nbins must be in 1..512");
  if (flags & ~(LPT2_POWER_DECONVOLVE | LPT2_POWER_INTERLACE)) return fail(p, LPT2_EINVAL, "unknown flags");
  const bool deconvolve = (flags & LPT2_POWER_DECONVOLVE) != 0, interlace = (flags & LPT2_POWER_INTERLACE) != 0;
  hipStream_t s = (hipStream_t)stream;
  Grid& g = p->grids[p->rgrid[0]];
  Ctx c{p, g, s, 2 * p->es, p->ws, 1};
  // CIC density into slot k (as a real field, particles moved by `shift`
  // cells), its 3D forward transform in place
  auto density_k = [&](int k, double shift) -> lpt2_status {
    RUN("cic_paint", 7.0 * (double)c.field(),
        launch_cic(p->prec, g.n, g.cfg.box, psi1, psi2, c.slot(k), s, shift));
    CHK(fwd_zy(c, "z_r2c_density", "y_fwd_density", c.one(c.slot(k), 1), c.cap(c.slot(k)), c.slot(k)));
    RUN("x_fwd_density", 2.0 * (double)c.field(),
        launch_colfft(p->prec, g.n, -1, c.slot(k), c.cap(c.slot(k)), 1, 0, (int)(g.n * g.m), g.n * g.m, g.tw, s,
                      g.tiles[0]));
    return LPT2_OK;
  };
  CHK(density_k(0, 0.0));
  if (interlace) {  // the second painting half a cell over, combined into slot 0
    CHK(density_k(1, 0.5));
    RUN("interlace", 3.0 * (double)c.field(),
        launch_interlace(p->prec, g.n, c.slot(0), c.cap(c.slot(0)), c.slot(1), c.cap(c.slot(1)), s));
  }
  const double n3 = (double)g.n3, kf = 2.0 * kPi / g.cfg.box;
  const double qs = g.cfg.box * g.cfg.box * g.cfg.box / (n3 * n3);
  RUN("shell_bin", 0.0,
      launch_bin(p->prec, g.n, c.slot(0), c.cap(c.slot(0)), nullptr, 0, deconvolve ? 2 : 0, qs, nbins, kf,
                 p->bin_partial, p->bin_out, s));
  std::vector<double> h(4 * (size_t)nbins);
  hipError_t e = hipMemcpyAsync(h.data(), p->bin_out, sizeof(double) * 4 * nbins, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(p, e, "spectrum readback");
  for (int i = 0; i < nbins; ++i) {
    k_mean[i] = h[i];
    count[i] = h[nbins + i];
    mean[i] = h[2 * nbins + i];
    std_dev[i] = h[3 * nbins + i];
  }
  return LPT2_OK;
}

lpt2_status lpt2_positions(lpt2_plan_t p, int r, const void* psi1, const void* psi2, void* pos, void* stream) {
  if (!p) return fail(nullptr, LPT2_EINVAL, "plan is NULL");
  if (r < 0 || r >= (int)p->rgrid.size()) return fail(p, LPT2_EINVAL, "realisation index out of range");
  if (!psi1 || !psi2 || !pos) return fail(p, LPT2_EINVAL, "null pointer");
  const Grid& g = p->grids[p->rgrid[r]];
  hipStream_t s = (hipStream_t)stream;
  RUN("positions", 9.0 * (double)g.n3 * p->es,
      launch_positions(p->prec, g.n, g.cfg.box, psi1, psi2, pos, s));
  return LPT2_OK;
}

lpt2_status lpt2_check_finite(lpt2_plan_t p, const void* field, long long count, long long* nonfinite,
                              void* stream) {
  if (!p) return fail(nullptr, LPT2_EINVAL, "plan is NULL");
  Busy b(p);
  if (!b.ok) return fail(p, LPT2_ESTATE, "plan is in use by another call");
  if (!field || !nonfinite || count < 0) return fail(p, LPT2_EINVAL, "null pointer or negative count");
  *nonfinite = 0;
  if (count == 0) return LPT2_OK;
  hipStream_t s = (hipStream_t)stream;
  RUN("check_finite", (double)count * p->es, launch_count_nonfinite(p->prec, field, count, p->counter, s));
  unsigned long long h = 0;
  hipError_t e = hipMemcpyAsync(&h, p->counter, sizeof(h), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(p, e, "counter readback");
  *nonfinite = (long long)h;
  if (h) return fail(p, LPT2_EINVAL, std::to_string(h) + " non-finite values");
  return LPT2_OK;
}

lpt2_status lpt2_backward(lpt2_plan_t p, double a, const void* const* noise, const void* const* g_psi1,
                          const void* const* g_psi2, void* const* g_noise, void* stream) {
  if (!p) return fail(nullptr, LPT2_EINVAL, "plan is NULL");
  Busy b(p);
  if (!b.ok) return fail(p, LPT2_ESTATE, "plan is in use by another call");
  CHK(check_a(p, a));
  if (!noise || !g_psi1 || !g_psi2 || !g_noise) return fail(p, LPT2_EINVAL, "null pointer array");
  const int nr = (int)p->rgrid.size();
  for (int r = 0; r < nr; ++r)
    if (!noise[r] || !g_psi1[r] || !g_psi2[r] || !g_noise[r])
      return fail(p, LPT2_EINVAL, "null field pointer for realisation " + std::to_string(r));
  hipStream_t s = (hipStream_t)stream;
  for (auto& g : p->grids) CHK(resolve_auto(p, g, a, noise[g.rfirst], s));
  for (int r = 0; r < nr; ++r) {
    Grid& g = p->grids[p->rgrid[r]];
    Tables* t = nullptr;
    CHK(get_tables(p, g, a, false, s, &t));
    Ctx c{p, g, s, 2 * p->es, p->ws, 1};
    CHK(backward_one(c, t, noise[r], g_psi1[r], g_psi2[r], g_noise[r]));
  }
  return LPT2_OK;
}

lpt2_status lpt2_paint_cic(lpt2_plan_t p, const void* psi1, const void* psi2, void* delta, void* stream) {
  if (!p) return fail(nullptr, LPT2_EINVAL, "plan is NULL");
  Busy b(p);
  if (!b.ok) return fail(p, LPT2_ESTATE, "plan is in use by another call");
  if (!psi1 || !psi2 || !delta) return fail(p, LPT2_EINVAL, "null pointer");
  hipStream_t s = (hipStream_t)stream;
  Grid& g = p->grids[p->rgrid[0]];
  RUN("cic_paint", 0.0, launch_cic(p->prec, g.n, g.cfg.box, psi1, psi2, delta, s));
  return LPT2_OK;
}

lpt2_status lpt2_paint_cic_backward(lpt2_plan_t p, const void* psi1, const void* psi2, const void* g_delta, void* g_psi,
                                    void* stream) {
  if (!p) return fail(nullptr, LPT2_EINVAL, "plan is NULL");
  Busy b(p);
  if (!b.ok) return fail(p, LPT2_ESTATE, "plan is in use by another call");
  if (!psi1 || !psi2 || !g_delta || !g_psi) return fail(p, LPT2_EINVAL, "null pointer");
  hipStream_t s = (hipStream_t)stream;
  Grid& g = p->grids[p->rgrid[0]];
  RUN("cic_backward", 0.0, launch_cic_back(p->prec, g.n, g.cfg.box, psi1, psi2, g_delta, g_psi, s));
  return LPT2_OK;
}

lpt2_status lpt2_growth_table(lpt2_plan_t p, double a, double* k, double* d1, double* d2) {
  if (!p) return fail(nullptr, LPT2_EINVAL, "plan is NULL");
  Busy b(p);
  if (!b.ok) return fail(p, LPT2_ESTATE, "plan is in use by another call");
  CHK(check_a(p, a));
  if (!k || !d1 || !d2) return fail(p, LPT2_EINVAL, "null pointer");
  Grid& g = p->grids[p->rgrid[0]];
  if (g.cfg.factorisation == LPT2_D2_AUTO && auto_lookup(g, a) == kAutoNone)
    return fail(p, LPT2_ESTATE, "AUTO factorisation not chosen at this a (run lpt2_displace or "
                                "lpt2_choose_factorisation first)");
  Tables* t = nullptr;
  CHK(get_tables(p, g, a, false, nullptr, &t));
  const int n = g.cfg.nk_growth;
  hipError_t e = hipMemcpy(d1, t->d1n, sizeof(double) * n, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(d2, t->d2n, sizeof(double) * n, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(p, e, "growth readback");
  for (int i = 0; i < n; ++i) k[i] = std::exp(g.lkmin + (g.lkmax - g.lkmin) * (double)i / (double)(n - 1));
  return LPT2_OK;
}

lpt2_status lpt2_fft3d(lpt2_plan_t p, int direction, const void* in, void* out, void* stream) {
  if (!p) return fail(nullptr, LPT2_EINVAL, "plan is NULL");
  Busy b(p);
  if (!b.ok) return fail(p, LPT2_ESTATE, "plan is in use by another call");
  if (!in || !out) return fail(p, LPT2_EINVAL, "null pointer");
  if (direction != -1 && direction != 1) return fail(p, LPT2_EINVAL, "direction must be -1 or +1");
  hipStream_t s = (hipStream_t)stream;
  Grid& g = p->grids[p->rgrid[0]];
  Ctx c{p, g, s, 2 * p->es, p->ws, 1};
  const double fb = (double)g.n3 * p->es;
  if (direction < 0) {
    RUN("z_r2c", 2.0 * fb, launch_zr2c(p->prec, g.n, c.one(in, 1), c.field(), out, c.field(), g.tw, s));
    RUN("y_fwd", 2.0 * fb,
        launch_colfft(p->prec, g.n, -1, out, c.field(), g.n, g.n * g.m, (int)g.m, g.m, g.tw, s));
    RUN("x_fwd", 2.0 * fb,
        launch_colfft(p->prec, g.n, -1, out, c.field(), 1, 0, (int)(g.n * g.m), g.n * g.m, g.tw, s));
  } else {
    hipError_t e = hipMemcpyAsync(c.slot(0), in, c.field(), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(p, e, "copy");
    RUN("x_inv", 2.0 * fb,
        launch_colfft(p->prec, g.n, +1, c.slot(0), c.cap(c.slot(0)), 1, 0, (int)(g.n * g.m), g.n * g.m, g.tw, s));
    CHK(inv_y(c, "y_inv", c.slot(0), 1));
    CHK(z_c2r(c, "z_c2r", c.slot(0), c.one(out, 1), c.field()));
  }
  return LPT2_OK;
}

lpt2_status lpt2_profile_enable(lpt2_plan_t p, int enable) {
  if (!p) return fail(nullptr, LPT2_EINVAL, "plan is NULL");
  prof_flush(p);
  p->prof = enable != 0;
  return LPT2_OK;
}
lpt2_status lpt2_profile_reset(lpt2_plan_t p) {
  if (!p) return fail(nullptr, LPT2_EINVAL, "plan is NULL");
  prof_flush(p);
  p->prof_tab.clear();
  return LPT2_OK;
}
int lpt2_profile_count(lpt2_plan_t p) {
  if (!p) return 0;
  prof_flush(p);
  return (int)p->prof_tab.size();
}
lpt2_status lpt2_profile_get(lpt2_plan_t p, int i, const char** name, long long* launches, double* total_ms,
                             double* bytes_per_launch) {
  if (!p) return fail(nullptr, LPT2_EINVAL, "plan is NULL");
  prof_flush(p);
  if (i < 0 || i >= (int)p->prof_tab.size()) return fail(p, LPT2_EINVAL, "profile index out of range");
  const ProfEntry& e = p->prof_tab[i];
  if (name) *name = e.name;
  if (launches) *launches = e.launches;
  if (total_ms) *total_ms = e.ms;
  if (bytes_per_launch) *bytes_per_launch = e.bytes;
  return LPT2_OK;
}

}  // extern "C"
