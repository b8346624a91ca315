// Simulation object: device workspace layout, table upload, the recursive
// multilevel schedule (Sec. 2.2) and the C ABI of the forward path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "kernels.hpp"
#include "launch.hpp"
#include "plan.hpp"
#include "sim.hpp"

namespace mlbm {

// Scratch of mlbm_diagnostics_noalloc: the per-block FP64 partials of the
// diagnostics reductions for up to DIAG_STATIC_LEVELS levels, in a
// file-scope device array (one copy per GPU, held until the process ends).
// Host code never passes the array's name to a kernel: it is a host-side
// stand-in there.  Its device address on each GPU comes from
// hipGetSymbolAddress, taken once per device (scratch_on_device).
constexpr int DIAG_STATIC_LEVELS = 16;
constexpr size_t DIAG_STATIC_DOUBLES = (size_t)DIAG_STATIC_LEVELS * DIAG_BLOCKS * DIAG_VALS;
static __device__ __align__(256) double scratch[DIAG_STATIC_DOUBLES];

namespace {

constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex scratch_mu;
double* scratch_ptr[SCRATCH_MAX_DEVICES] = {};

// Device address of `scratch` on `device` (which must be current); looked up
// on the first call per device.  Returns nullptr and sets *err on failure.
double* scratch_on_device(int device, hipError_t* err) {
  *err = hipSuccess;
  if (device < 0 || device >= SCRATCH_MAX_DEVICES) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (!scratch_ptr[device]) {
    void* p = nullptr;
    *err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (*err != hipSuccess) return nullptr;
    scratch_ptr[device] = (double*)p;
  }
  return scratch_ptr[device];
}

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

size_t storage_bytes(int precision) {
  return precision == MLBM_F64 ? 8 : (precision == MLBM_F32 ? 4 : 2);
}
size_t compute_bytes(int precision) { return precision == MLBM_F64 ? 8 : 4; }

}  // namespace

// Carves the workspace; with base == nullptr only the size is computed.
size_t layout_workspace(const mlbm_plan& P, int precision, char* base, SimState* s) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += align_up(bytes);
    return p;
  };
  const int d = P.d, q = P.q;
  const size_t sb = storage_bytes(precision), cb = compute_bytes(precision);
  const int NB = group_slots(d), NC = group_children(d);
  for (int k = 0; k < P.nlev(); ++k) {
    const auto& lp = P.lv[k];
    DevLevel* L = s ? &s->lv[k] : nullptr;
    const int64_t ld = row_stride(lp.n);
    char* p0 = take((size_t)q * ld * sb);
    char* p1 = take((size_t)q * ld * sb);
    char* n16 = take(lp.nbr16.size() * 2);
    char* nbs = take(lp.nbase.size() * 4);
    char* nwd = take(lp.nbr_wide.size() * 2);
    char* nhd = take(lp.nhdr.size() * 4);
    char* ce = take((size_t)lp.n_cap_fluid() * 4);
    char* cap = take((size_t)lp.n_cap() * cap_stride(q) * cb);
    char* gs = take((size_t)4 * lp.n_gff * 4);
    char* grs = take((size_t)NB * lp.n_groups * 4);
    char* grt = take(lp.grp_tab.size() * 4);
    char* grc = take((size_t)NC * lp.n_groups * 4);
    char* bb = take((size_t)2 * lp.n_bounce() * 4);
    char* wl = take(lp.wall_dev.size() * 4);
    char* wq = take(lp.wall_dev_q.size() * 8);
    if (L) {
      L->pdf[0] = p0;
      L->pdf[1] = p1;
      L->nbr16 = (uint16_t*)n16;
      L->nbase = (int32_t*)nbs;
      L->nbr_wide = (uint16_t*)nwd;
      L->nhdr = (int32_t*)nhd;
      L->ld16 = lp.n_nbr_blocks() * NBR_BLOCK;
      L->ldw = lp.n_wide * NBR_BLOCK;
      L->cap_elem = (int32_t*)ce;
      L->cap = cap;
      L->gff_slot = (int32_t*)gs;
      L->grp_src = (int32_t*)grs;
      L->grp_tab = (int32_t*)grt;
      L->grp_child = (int32_t*)grc;
      L->bounce = (int32_t*)bb;
      L->wall = lp.n_wall() ? (int32_t*)wl : nullptr;
      L->wall_q = lp.n_wall() ? (double*)wq : nullptr;
    }
  }
  char* st = take(256);
  char* part = take((size_t)P.nlev() * DIAG_BLOCKS * DIAG_VALS * 8);
  char* dl = take((size_t)P.nlev() * sizeof(DiagLevel));
  char* md = take(256 * 8);
  char* gq = take((size_t)q * cb);
  if (s) {
    s->status = (uint32_t*)st;
    s->partial = (double*)part;
    s->diag_levels = dl;
    s->maxdev = (double*)md;
    s->geq_dev = gq;
  }
  return off;
}

void SimState::drop_graphs() {
  for (auto& g : graphs) (void)hipGraphExecDestroy(g.second);
  graphs.clear();
}

SimState::~SimState() {
  drop_graphs();
  for (hipEvent_t e : prof.pool) (void)hipEventDestroy(e);
  if (capture_stream) (void)hipStreamDestroy(capture_stream);
  if (adj.fork) (void)hipEventDestroy(adj.fork);
  if (adj.join) (void)hipEventDestroy(adj.join);
  if (adj.side) (void)hipStreamDestroy(adj.side);
}

hipEvent_t prof_event(SimState& s) {
  if (s.prof.used == s.prof.pool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    s.prof.pool.push_back(e);
  }
  return s.prof.pool[s.prof.used++];
}

// Launches the pending stream-collides (one per level) as one grid.
void flush_sc(SimState& s) {
  if (s.pending.empty()) return;
  MLBM_DISPATCH(s, I::stream_collide_multi(s, s.pending.data(), (int)s.pending.size()));
  s.pending.clear();
}

// Launches the pending fills (consecutive fills of different level pairs)
// as one grid.
void flush_fill(SimState& s) {
  if (s.pending_fill.empty()) return;
  MLBM_DISPATCH(s, I::fill_sync_multi(s, s.pending_fill.data(), (int)s.pending_fill.size()));
  s.pending_fill.clear();
}

// Active set of a stream-collide of level k > 0: fluid, plus the inner
// GhostFromCoarser layers on every step after a sync but the last of the
// parent's step.  With n_sub = 2 (one inner layer) that is the first step.
// With n_sub = 4 the inner layers are at distances 1-3 from fluid: the fluid
// reads layer 1 at each step, which needs layer 2 one step and layer 3 two
// steps earlier, and layer 3 reads the outer layer filled at the sync.  The
// whole inner part is updated on the first three steps; values of the deeper
// layers past what the fluid needs are never read by it.
static int64_t active_count(const SimState& s, const DevLevel& L, int k) {
  const bool inner = (k > 0) && (L.substep < s.n_sub - 1);
  return L.n_fluid + (inner ? L.n_inner : 0);
}

void sc_level(SimState& s, int k) {
  DevLevel& L = s.lv[k];
  const int64_t n_act = active_count(s, L, k);
  flush_fill(s);   // a stream-collide reads the ghosts the fills write
  if (!s.prof.on) {
    // consecutive stream-collides of different levels share a launch; a
    // second one of the same level depends on the first
    for (const auto& j : s.pending)
      if (j.k == k) {
        flush_sc(s);
        break;
      }
    if ((int)s.pending.size() == SC_MAX_SEG) flush_sc(s);
    s.pending.push_back(ScJob{k, n_act, L.pdf[L.parity], L.pdf[L.parity ^ 1], L.cap});
    L.parity ^= 1;
    if (k > 0) L.substep = (L.substep + 1) % s.n_sub;
    return;
  }
  flush_sc(s);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (s.prof.on && n_act > 0) {
    e0 = prof_event(s);
    e1 = prof_event(s);
    if (e0 && e1) {
      s.launch_ev[0] = e0;
      s.launch_ev[1] = e1;
    }
  }
  MLBM_DISPATCH(s, I::stream_collide(s, k, n_act));
  s.launch_ev[0] = s.launch_ev[1] = nullptr;
  if (s.prof.on && e0 && e1) s.prof.rec.push_back({0, k, n_act, e0, e1});
  L.parity ^= 1;
  if (k > 0) L.substep = (L.substep + 1) % s.n_sub;
}

void fill_gff(SimState& s, int k) { MLBM_DISPATCH(s, I::fill_gff(s, k)); }
void fill_sync(SimState& s, int k) {
  flush_sc(s);   // the fills read the records the stream-collides write
  if (s.prof.on) {
    flush_fill(s);
    MLBM_DISPATCH(s, I::fill_sync(s, k));
    return;
  }
  for (const auto& j : s.pending_fill)
    if (j.k == k) {
      flush_fill(s);
      break;
    }
  if ((int)s.pending_fill.size() == FILL_MAX_SEG) flush_fill(s);
  DevLevel& L = s.lv[k];
  DevLevel& F = s.lv[k + 1];
  s.pending_fill.push_back(FillJob{k, L.pdf[L.parity], F.cap, L.cap, F.pdf[F.parity]});
}
void fill_gfc(SimState& s, int k) { MLBM_DISPATCH(s, I::fill_gfc(s, k)); }

void advance(SimState& s, int k) {
  sc_level(s, k);
  if (k + 1 < (int)s.lv.size()) {
    for (int t = 0; t < s.n_sub; ++t) advance(s, k + 1);
    fill_sync(s, k);   // GhostFromFiner(k) and GhostFromCoarser(k+1)
  }
}

static uint64_t parity_key(const SimState& s) {
  uint64_t key = 0;
  for (size_t k = 0; k < s.lv.size() && k < 21; ++k)
    key |= (uint64_t)(s.lv[k].parity & 1) << (3 * k) | (uint64_t)(s.lv[k].substep & 3) << (3 * k + 1);
  return key;
}

// Records two coarse steps into a graph on the capture stream.  Every level
// takes an even number of stream-collides in two coarse steps, a multiple of
// n_sub below the coarsest, so the parity and substep state after the graph
// equals the state it was captured from.
static hipError_t two_step_graph(SimState& s, hipGraphExec_t* exec) {
  hipError_t e = hipSuccess;
  if (!s.capture_stream) e = hipStreamCreateWithFlags(&s.capture_stream, hipStreamNonBlocking);
  if (e != hipSuccess) return e;
  const hipStream_t user = s.stream;
  std::vector<std::pair<int, int>> saved;
  for (auto& L : s.lv) saved.emplace_back(L.parity, L.substep);
  s.stream = s.capture_stream;
  e = hipStreamBeginCapture(s.stream, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    advance(s, 0);
    advance(s, 0);
    flush_sc(s);
    flush_fill(s);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(s.stream, &graph);
    if (e == hipSuccess) e = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
  }
  s.stream = user;
  for (size_t k = 0; k < s.lv.size(); ++k) {
    s.lv[k].parity = saved[k].first;
    s.lv[k].substep = saved[k].second;
  }
  return e;
}

int32_t check_launch(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(MLBM_E_HIP, "%s: %s", what, hipGetErrorString(e));
  return MLBM_OK;
}

}  // namespace mlbm

using namespace mlbm;

extern "C" {

int32_t mlbm_sim_workspace_bytes(const mlbm_plan* plan, int32_t precision, size_t* bytes) {
  if (!plan || !bytes) return fail(MLBM_E_ARG, "NULL argument");
  if (precision < MLBM_F64 || precision > MLBM_F16S) return fail(MLBM_E_ARG, "bad precision");
  *bytes = layout_workspace(*plan, precision, nullptr, nullptr);
  return MLBM_OK;
}

int32_t mlbm_sim_create(const mlbm_plan* plan, int32_t precision, double tau0, double rho0,
                        const double* u_in, const int32_t* f16_exp, void* hip_stream,
                        void* workspace, size_t workspace_bytes, mlbm_sim** out) {
  if (!out) return fail(MLBM_E_ARG, "out is NULL");
  *out = nullptr;
  if (!plan || !workspace) return fail(MLBM_E_ARG, "NULL plan or workspace");
  if (precision < MLBM_F64 || precision > MLBM_F16S) return fail(MLBM_E_ARG, "bad precision");
  if (!(tau0 > 0.5)) return fail(MLBM_E_ARG, "tau0 must exceed 1/2");
  if (!(rho0 > 0.0)) return fail(MLBM_E_ARG, "rho0 must be positive");
  if (((uintptr_t)workspace) & 255) return fail(MLBM_E_ARG, "workspace must be 256-byte aligned");
  // the stream-collide addresses a pair of pdf rows (and a neighbour row)
  // through one buffer descriptor with 32-bit byte offsets
  const size_t pdf_bytes = precision == MLBM_F64 ? 8 : precision == MLBM_F32 ? 4 : 2;
  for (const auto& lp : plan->lv)
    if ((uint64_t)row_stride(lp.n) * pdf_bytes * 2 >= (1ull << 32) || (uint64_t)lp.n * 4 >= (1ull << 32))
      return fail(MLBM_E_ARG,
                  "level %d has %lld elements: two pdf rows must stay below 4 GiB",
                  lp.level, (long long)lp.n);
  const size_t need = layout_workspace(*plan, precision, nullptr, nullptr);
  if (workspace_bytes < need)
    return fail(MLBM_E_ARG, "workspace too small: need %zu bytes, got %zu", need, workspace_bytes);
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) return fail(MLBM_E_HIP, "no current HIP device");
  {
    // the no-allocation diagnostics' scratch: its address on this device
    hipError_t se = hipSuccess;
    if (!scratch_on_device(device, &se))
      return fail(MLBM_E_HIP, "scratch address on device %d: %s", device, hipGetErrorString(se));
  }
  mlbm_sim* sim = new (std::nothrow) mlbm_sim();
  if (!sim) return fail(MLBM_E_OOM, "host allocation failed");
  SimState& s = sim->s;
  s.device = device;
  s.n_sub = plan->gfc_layers == 4 ? 4 : 2;   // four layers: diffusive scaling
  s.stencil = plan->stencil;
  s.d = plan->d;
  s.q = plan->q;
  s.precision = precision;
  s.level0 = plan->level0;
  s.tau0 = tau0;
  s.rho0 = rho0;
  s.stream = (hipStream_t)hip_stream;
  s.ws = (char*)workspace;
  s.ws_bytes = workspace_bytes;
  for (int a = 0; a < 3; ++a) s.u_in[a] = (u_in && a < s.d) ? u_in[a] : 0.0;
  s.lv.resize(plan->nlev());
  for (int k = 0; k < plan->nlev(); ++k) {
    const auto& lp = plan->lv[k];
    DevLevel& L = s.lv[k];
    L.level = lp.level;
    L.n = lp.n;
    L.ld = row_stride(lp.n);
    L.n_fluid = lp.n_fluid;
    L.n_inner = lp.n_inner;
    L.n_outer = lp.n_outer;
    L.n_gff = lp.n_gff;
    L.n_act_max = lp.n_active_max();
    L.n_cap_fluid = lp.n_cap_fluid();
    L.n_cap = lp.n_cap();
    L.n_groups = lp.n_groups;
    L.n_bounce = lp.n_bounce();
    L.n_wall = lp.n_wall_dev();
    L.morton = lp.morton;
    // acoustic scaling: Eq. fneq_scale per level jump (tau_L - 1/2 doubles);
    // diffusive scaling: nu dt / dx^2 is level invariant, one tau everywhere
    const double tau = s.n_sub == 4 ? tau0 : 0.5 + std::ldexp(tau0 - 0.5, lp.level - plan->level0);
    L.omega = 1.0 / tau;
    L.f16_exp = f16_exp ? f16_exp[k] : 0;
    L.f16_auto = (f16_exp == nullptr) && precision == MLBM_F16S;
  }
  // lattice constants: w_i rho0 and the EQ-face equilibrium deviation
  for (int i = 0; i < s.q; ++i) {
    const double w = stencil_w(s.stencil, i);
    double cu = 0, uu = 0;
    for (int a = 0; a < s.d; ++a) cu += stencil_c(s.stencil, i, a) * s.u_in[a];
    for (int a = 0; a < s.d; ++a) uu += s.u_in[a] * s.u_in[a];
    s.wr[i] = w * rho0;
    s.geq[i] = w * rho0 * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
  }
  layout_workspace(*plan, precision, s.ws, &s);
  // upload tables
  hipError_t e = hipSuccess;
  auto up = [&](void* dst, const void* src, size_t bytes) {
    if (bytes && e == hipSuccess) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s.stream);
  };
  for (int k = 0; k < plan->nlev() && e == hipSuccess; ++k) {
    const auto& lp = plan->lv[k];
    DevLevel& L = s.lv[k];
    up(L.nbr16, lp.nbr16.data(), lp.nbr16.size() * 2);
    up(L.nbase, lp.nbase.data(), lp.nbase.size() * 4);
    up(L.nbr_wide, lp.nbr_wide.data(), lp.nbr_wide.size() * 2);
    up(L.nhdr, lp.nhdr.data(), lp.nhdr.size() * 4);
    up(L.cap_elem, lp.cap_elem.data(), lp.cap_elem.size() * 4);
    up(L.gff_slot, lp.gff_slot.data(), lp.gff_slot.size() * 4);
    up(L.grp_src, lp.grp_src.data(), lp.grp_src.size() * 4);
    up(L.grp_tab, lp.grp_tab.data(), lp.grp_tab.size() * 4);
    up(L.grp_child, lp.grp_child.data(), lp.grp_child.size() * 4);
    up(L.bounce, lp.bounce.data(), lp.bounce.size() * 4);
    up(L.wall, lp.wall_dev.data(), lp.wall_dev.size() * 4);
    up(L.wall_q, lp.wall_dev_q.data(), lp.wall_dev_q.size() * 8);
  }
  std::vector<DiagLevel> dl(plan->nlev());
  for (int k = 0; k < plan->nlev(); ++k) {
    const int L = plan->lv[k].level;
    dl[k].vol = std::ldexp(1.0, -s.d * (L - plan->level0));
    dl[k].force_scale = std::ldexp(1.0, (s.d - 1) * (plan->level0 + plan->nlev() - 1 - L));
    dl[k].rho0_nf = rho0 * (double)plan->lv[k].n_fluid;
    // level-L0 units of velocity and density deviation: u dt/dx and
    // (rho - rho0) dt^2/dx^2 grow by n_sub/2 and its square per level
    dl[k].unit2 = std::pow(0.5 * s.n_sub, 2.0 * (L - plan->level0));
  }
  up(s.diag_levels, dl.data(), dl.size() * sizeof(DiagLevel));
  std::vector<double> geq_d(s.geq, s.geq + s.q);
  std::vector<float> geq_f(s.geq, s.geq + s.q);
  if (compute_bytes(precision) == 8)
    up(s.geq_dev, geq_d.data(), geq_d.size() * 8);
  else
    up(s.geq_dev, geq_f.data(), geq_f.size() * 4);
  if (e == hipSuccess) e = hipMemsetAsync(s.status, 0, 256, s.stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s.stream);
  if (e != hipSuccess) {
    delete sim;
    return fail(MLBM_E_HIP, "table upload: %s", hipGetErrorString(e));
  }
  s.inited.assign(plan->nlev(), false);
  *out = sim;
  return MLBM_OK;
}

void mlbm_sim_destroy(mlbm_sim* sim) { delete sim; }

int32_t mlbm_init(mlbm_sim* sim, int32_t k, const double* rho, const double* u, const double* S) {
  if (!sim) return fail(MLBM_E_ARG, "sim is NULL");
  SimState& s = sim->s;
  if (k < 0 || k >= (int)s.lv.size()) return fail(MLBM_E_ARG, "level index %d out of range", k);
  DevLevel& L = s.lv[k];
  if (L.n_fluid && (!rho || !u)) return fail(MLBM_E_ARG, "rho and u are required");
  if (L.f16_auto) {
    double m = 0;
    MLBM_DISPATCH(s, m = I::init_maxdev(s, k, rho, u, S));
    if (m < 0) return fail(MLBM_E_HIP, "FP16 scale reduction failed");
    // largest power of two with max|f - w rho0| * s_L <= 2^12
    int ex = m > 0 ? (int)std::floor(std::log2(4096.0 / m)) : 24;
    L.f16_exp = std::min(24, std::max(0, ex));
  }
  s.drop_graphs();
  MLBM_DISPATCH(s, I::init(s, k, rho, u, S));
  L.parity = 0;
  L.substep = 0;
  L.pre_valid = false;
  s.inited[k] = true;
  s.time = 0;
  return check_launch("mlbm_init");
}

int32_t mlbm_fill_ghosts(mlbm_sim* sim) {
  if (!sim) return fail(MLBM_E_ARG, "sim is NULL");
  SimState& s = sim->s;
  for (bool b : s.inited)
    if (!b) return fail(MLBM_E_STATE, "mlbm_init must be called for every level first");
  for (int k = 0; k + 1 < (int)s.lv.size(); ++k) fill_gff(s, k);
  for (int k = 1; k < (int)s.lv.size(); ++k) fill_gfc(s, k);
  s.filled = true;
  return check_launch("mlbm_fill_ghosts");
}

int32_t mlbm_step(mlbm_sim* sim, int64_t n_coarse) {
  if (!sim) return fail(MLBM_E_ARG, "sim is NULL");
  if (n_coarse < 0) return fail(MLBM_E_ARG, "negative step count");
  SimState& s = sim->s;
  if (!s.filled) return fail(MLBM_E_STATE, "mlbm_fill_ghosts must follow mlbm_init");
  int64_t left = n_coarse;
  if (s.use_graphs && !s.prof.on) {
    while (left >= 2) {
      const uint64_t key = parity_key(s);
      hipGraphExec_t exec = nullptr;
      for (auto& g : s.graphs)
        if (g.first == key) exec = g.second;
      if (!exec) {
        const hipError_t e = two_step_graph(s, &exec);
        if (e != hipSuccess) {
          (void)hipGetLastError();
          s.use_graphs = false;  // fall back to direct launches
          s.graph_fallback = true;
          break;
        }
        s.graphs.emplace_back(key, exec);
      }
      const hipError_t e = hipGraphLaunch(exec, s.stream);
      if (e != hipSuccess) return fail(MLBM_E_HIP, "graph launch: %s", hipGetErrorString(e));
      left -= 2;
      s.time += 2;
    }
  }
  for (; left > 0; --left) {
    advance(s, 0);
    s.time++;
  }
  flush_sc(s);
  flush_fill(s);
  if (n_coarse > 0)
    for (auto& L : s.lv) L.pre_valid = true;
  return check_launch("mlbm_step");
}

int32_t mlbm_diagnostics(mlbm_sim* sim, uint32_t mask, double* dev_out) {
  if (!sim || !dev_out) return fail(MLBM_E_ARG, "NULL argument");
  SimState& s = sim->s;
  if (!s.filled) return fail(MLBM_E_STATE, "no state yet");
  if (mask & ~7u) return fail(MLBM_E_ARG, "bad diagnostics mask");
  if ((mask & MLBM_DIAG_FORCE) && s.n_sub != 2)
    return fail(MLBM_E_STATE, "the force is defined for acoustic scaling only");
  for (int k = 0; k < (int)s.lv.size(); ++k) MLBM_DISPATCH(s, I::diag_partial(s, k));
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(256), 0, s.stream, s.partial, (int)s.lv.size(),
                     (const DiagLevel*)s.diag_levels, mask, s.d, dev_out);
  return check_launch("mlbm_diagnostics");
}

int32_t mlbm_diagnostics_noalloc(mlbm_sim* sim, uint32_t mask, double* dev_out) {
  if (!sim || !dev_out) return fail(MLBM_E_ARG, "NULL argument");
  SimState& s = sim->s;
  if (!s.filled) return fail(MLBM_E_STATE, "no state yet");
  if (mask & ~7u) return fail(MLBM_E_ARG, "bad diagnostics mask");
  if ((mask & MLBM_DIAG_FORCE) && s.n_sub != 2)
    return fail(MLBM_E_STATE, "the force is defined for acoustic scaling only");
  if ((int)s.lv.size() > DIAG_STATIC_LEVELS)
    return fail(MLBM_E_ARG, "%d levels: the static scratch holds the partials of at most %d",
                (int)s.lv.size(), DIAG_STATIC_LEVELS);
  hipError_t se = hipSuccess;
  double* part = scratch_on_device(s.device, &se);
  if (!part) return fail(MLBM_E_HIP, "scratch address: %s", hipGetErrorString(se));
  // every partial the final pass reads is written by this call's first
  // pass (a fixed grid of DIAG_BLOCKS work-groups per level): nothing to clear
  for (int k = 0; k < (int)s.lv.size(); ++k)
    MLBM_DISPATCH(s, I::diag_partial_to(s, k, part + (size_t)k * DIAG_BLOCKS * DIAG_VALS));
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(256), 0, s.stream, (const double*)part,
                     (int)s.lv.size(), (const DiagLevel*)s.diag_levels, mask, s.d, dev_out);
  return check_launch("mlbm_diagnostics_noalloc");
}

int32_t mlbm_get_state(mlbm_sim* sim, int32_t k, int32_t what, double* dev_dst) {
  if (!sim || !dev_dst) return fail(MLBM_E_ARG, "NULL argument");
  SimState& s = sim->s;
  if (k < 0 || k >= (int)s.lv.size()) return fail(MLBM_E_ARG, "level index %d out of range", k);
  if (what < MLBM_STATE_PDF_POST || what > MLBM_STATE_PDF_PREV)
    return fail(MLBM_E_ARG, "unknown state selector %d", what);
  if (!s.inited[k]) return fail(MLBM_E_STATE, "level %d has no state yet", k);
  DevLevel& L = s.lv[k];
  if (what >= MLBM_STATE_PDF_PRE && !L.pre_valid)
    return fail(MLBM_E_STATE, "level %d: no stream-collide since the state was last set "
                              "(init, set_state or load_checkpoint)", k);
  if (what == MLBM_STATE_PDF_POST) MLBM_DISPATCH(s, I::get_pdf(s, k, dev_dst));
  else if (what == MLBM_STATE_MOMENTS) MLBM_DISPATCH(s, I::get_moments(s, k, dev_dst));
  else if (what == MLBM_STATE_PDF_PRE) MLBM_DISPATCH(s, I::get_pulled(s, k, 0, dev_dst));
  else if (what == MLBM_STATE_STRAIN) MLBM_DISPATCH(s, I::get_pulled(s, k, 1, dev_dst));
  else MLBM_DISPATCH(s, I::get_prev(s, k, dev_dst));
  return check_launch("mlbm_get_state");
}

int32_t mlbm_set_state(mlbm_sim* sim, int32_t k, int32_t what, const double* dev_src) {
  if (!sim || !dev_src) return fail(MLBM_E_ARG, "NULL argument");
  SimState& s = sim->s;
  if (k < 0 || k >= (int)s.lv.size()) return fail(MLBM_E_ARG, "level index %d out of range", k);
  if (what != MLBM_STATE_PDF_POST && what != MLBM_STATE_PDF_PRE)
    return fail(MLBM_E_ARG, "set_state takes MLBM_STATE_PDF_POST or MLBM_STATE_PDF_PRE, not %d",
                what);
  if (what == MLBM_STATE_PDF_POST) MLBM_DISPATCH(s, I::set_pdf(s, k, dev_src));
  else MLBM_DISPATCH(s, I::set_pre(s, k, dev_src));
  s.drop_graphs();
  s.lv[k].pre_valid = false;
  s.inited[k] = true;
  return check_launch("mlbm_set_state");
}

int32_t mlbm_status(mlbm_sim* sim, uint32_t* flags) {
  if (!sim || !flags) return fail(MLBM_E_ARG, "NULL argument");
  SimState& s = sim->s;
  uint32_t h = 0;
  hipError_t e = hipMemcpyAsync(&h, s.status, 4, hipMemcpyDeviceToHost, s.stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s.stream);
  if (e == hipSuccess) e = hipMemsetAsync(s.status, 0, 4, s.stream);
  if (e != hipSuccess) return fail(MLBM_E_HIP, "status: %s", hipGetErrorString(e));
  if (s.graph_fallback) h |= MLBM_STATUS_GRAPH_FALLBACK;
  s.graph_fallback = false;
  *flags = h;
  return MLBM_OK;
}

int32_t mlbm_time(const mlbm_sim* sim, int64_t* coarse_steps) {
  if (!sim || !coarse_steps) return fail(MLBM_E_ARG, "NULL argument");
  *coarse_steps = sim->s.time;
  return MLBM_OK;
}

int32_t mlbm_checkpoint_bytes(const mlbm_sim* sim, size_t* bytes) {
  if (!sim || !bytes) return fail(MLBM_E_ARG, "NULL argument");
  const SimState& s = sim->s;
  size_t b = 256;
  for (const auto& L : s.lv) b += align_up((size_t)s.q * L.ld * storage_bytes(s.precision));
  *bytes = b;
  return MLBM_OK;
}

int32_t mlbm_save_checkpoint(mlbm_sim* sim, void* dev_dst, size_t bytes) {
  if (!sim || !dev_dst) return fail(MLBM_E_ARG, "NULL argument");
  SimState& s = sim->s;
  size_t need = 0;
  mlbm_checkpoint_bytes(sim, &need);
  if (bytes < need) return fail(MLBM_E_ARG, "checkpoint buffer too small (%zu < %zu)", bytes, need);
  if (!s.filled) return fail(MLBM_E_STATE, "no state to save");
  CheckpointHeader h{};
  h.magic = 0x4d4c424d43505431ull;
  h.time = s.time;
  h.nlev = (int32_t)s.lv.size();
  h.precision = s.precision;
  for (size_t k = 0; k < s.lv.size() && k < 16; ++k) h.f16_exp[k] = s.lv[k].f16_exp;
  char* p = (char*)dev_dst;
  hipError_t e = hipMemcpyAsync(p, &h, sizeof h, hipMemcpyHostToDevice, s.stream);
  size_t off = 256;
  for (auto& L : s.lv) {
    const size_t b = (size_t)s.q * L.ld * storage_bytes(s.precision);
    if (e == hipSuccess && b)
      e = hipMemcpyAsync(p + off, L.pdf[L.parity], b, hipMemcpyDeviceToDevice, s.stream);
    off += align_up(b);
  }
  // the header lives on the host stack: make sure it has been consumed
  if (e == hipSuccess) e = hipStreamSynchronize(s.stream);
  if (e != hipSuccess) return fail(MLBM_E_HIP, "save_checkpoint: %s", hipGetErrorString(e));
  return MLBM_OK;
}

int32_t mlbm_load_checkpoint(mlbm_sim* sim, const void* dev_src, size_t bytes) {
  if (!sim || !dev_src) return fail(MLBM_E_ARG, "NULL argument");
  SimState& s = sim->s;
  size_t need = 0;
  mlbm_checkpoint_bytes(sim, &need);
  if (bytes < need) return fail(MLBM_E_ARG, "checkpoint buffer too small (%zu < %zu)", bytes, need);
  CheckpointHeader h{};
  hipError_t e = hipMemcpyAsync(&h, dev_src, sizeof h, hipMemcpyDeviceToHost, s.stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s.stream);
  if (e != hipSuccess) return fail(MLBM_E_HIP, "load_checkpoint: %s", hipGetErrorString(e));
  if (h.magic != 0x4d4c424d43505431ull || h.nlev != (int32_t)s.lv.size() ||
      h.precision != s.precision)
    return fail(MLBM_E_ARG, "checkpoint does not belong to this simulation");
  const char* p = (const char*)dev_src;
  size_t off = 256;
  s.drop_graphs();
  for (size_t k = 0; k < s.lv.size(); ++k) {
    DevLevel& L = s.lv[k];
    const size_t b = (size_t)s.q * L.ld * storage_bytes(s.precision);
    L.parity = 0;
    L.substep = 0;
    L.pre_valid = false;
    if (k < 16) L.f16_exp = h.f16_exp[k];
    if (e == hipSuccess && b)
      e = hipMemcpyAsync(L.pdf[0], p + off, b, hipMemcpyDeviceToDevice, s.stream);
    off += align_up(b);
  }
  if (e != hipSuccess) return fail(MLBM_E_HIP, "load_checkpoint: %s", hipGetErrorString(e));
  s.time = h.time;
  std::fill(s.inited.begin(), s.inited.end(), true);
  s.filled = true;
  return MLBM_OK;
}

int32_t mlbm_use_graphs(mlbm_sim* sim, int32_t enable) {
  if (!sim) return fail(MLBM_E_ARG, "sim is NULL");
  sim->s.use_graphs = enable != 0;
  if (!enable) sim->s.drop_graphs();
  return MLBM_OK;
}

int32_t mlbm_profile(mlbm_sim* sim, int32_t enable) {
  if (!sim) return fail(MLBM_E_ARG, "sim is NULL");
  SimState& s = sim->s;
  if (enable) {
    if (hipStreamSynchronize(s.stream) != hipSuccess) return fail(MLBM_E_HIP, "profile: sync failed");
    s.prof.rec.clear();
    s.prof.used = 0;
  }
  s.prof.on = enable != 0;
  return MLBM_OK;
}

int32_t mlbm_profile_read(mlbm_sim* sim, int32_t k, double* ms, int64_t* launches,
                          int64_t* elements) {
  return mlbm_profile_read_kind(sim, 0, k, ms, launches, elements);
}

int32_t mlbm_profile_read_kind(mlbm_sim* sim, int32_t kind, int32_t k, double* ms,
                               int64_t* launches, int64_t* elements) {
  if (!sim || !ms || !launches || !elements) return fail(MLBM_E_ARG, "NULL argument");
  SimState& s = sim->s;
  if (k < 0 || k >= (int)s.lv.size()) return fail(MLBM_E_ARG, "level index %d out of range", k);
  if (hipStreamSynchronize(s.stream) != hipSuccess) return fail(MLBM_E_HIP, "profile: sync failed");
  double t = 0;
  int64_t n = 0, el = 0;
  for (const auto& r : s.prof.rec) {
    if (r.level != k || r.kind != kind) continue;
    float dt = 0;
    if (hipEventElapsedTime(&dt, r.start, r.stop) != hipSuccess)
      return fail(MLBM_E_HIP, "profile: elapsed time failed");
    t += dt;
    n++;
    el += r.n_act;
  }
  *ms = t;
  *launches = n;
  *elements = el;
  return MLBM_OK;
}

int32_t mlbm_launches_per_step(const mlbm_sim* sim, int64_t* launches) {
  if (!sim || !launches) return fail(MLBM_E_ARG, "NULL argument");
  const SimState& s = sim->s;
  int64_t total = 0;
  int64_t reps = 1;
  for (size_t k = 0; k < s.lv.size(); ++k, reps *= s.n_sub) {
    const auto& L = s.lv[k];
    total += reps;
    if (k + 1 < s.lv.size()) total += reps * ((L.n_gff || s.lv[k + 1].n_groups) ? 1 : 0);
  }
  *launches = total;
  return MLBM_OK;
}

}  // extern "C"
