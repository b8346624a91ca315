// Host-side simulation state shared by the forward and adjoint translation
// units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "common.hpp"

struct mlbm_plan;

namespace mlbm {

struct DevLevel {
  int level = 0;
  int64_t n = 0, n_fluid = 0, n_inner = 0, n_outer = 0, n_gff = 0, n_act_max = 0;
  int64_t ld = 0;                     // row stride of the [q][ld] pdf-like arrays
  int64_t n_cap_fluid = 0, n_cap = 0, n_groups = 0, n_bounce = 0, n_wall = 0;
  void* pdf[2] = {nullptr, nullptr};  // storage arrays [q][n]
  uint16_t* nbr16 = nullptr;          // pull table, device form: [q-1][ld16]
  int32_t* nbase = nullptr;           // [blocks][q-1][NBR_BASES]
  uint16_t* nbr_wide = nullptr;       // [q-1][ldw] high halves of wide blocks
  int32_t* nhdr = nullptr;            // [blocks][NBR_HDR]
  bool morton = false;                // blocks may hold Morton directions
  int64_t ld16 = 0, ldw = 0;
  int32_t* cap_elem = nullptr;        // [n_cap_fluid]
  void* cap = nullptr;                // [n_cap][cap_stride] compute type
  int32_t* gff_slot = nullptr;        // [4][n_gff] capture slots on level+1
  int32_t* grp_src = nullptr;         // [slots][n_groups] capture slots on level-1
  int32_t* grp_tab = nullptr;         // [slots][n_groups][4] fill staging rows
  int32_t* grp_child = nullptr;       // [children][n_groups] element indices
  int32_t* bounce = nullptr;          // [2][n_bounce]
  int32_t* wall = nullptr;            // [n_wall][4] links with a wall fraction,
  double* wall_q = nullptr;           // [n_wall]    padded (the plan's device copy)
  int parity = 0;                     // index of the current pdf array
  int substep = 0;                    // steps since the last sync (0: the first after one)
  bool pre_valid = false;             // the other array holds what the last
                                      // stream-collide read
  double omega = 1.0;
  int f16_exp = 0;
  bool f16_auto = false;
};

// Event-bracketed timing of stream-collide launches.
struct ProfRecord {
  int kind;   // 0: forward stream-collide, 1: adjoint stream-collide
  int level;
  int64_t n_act;
  hipEvent_t start, stop;
};
struct Profiler {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<ProfRecord> rec;
};

struct AdjOp;
struct AdjChunk;

// A stream-collide waiting to be launched together with those of other
// levels (see mlbm::flush_sc).
struct ScJob {
  int k;
  int64_t n_act;
  const void* src;
  void* dst;
  void* cap;
  int64_t x0 = 0;   // elements below the block of x0 are skipped (their
                    // results are not needed; see the adjoint's tape)
};
// A fill of levels (k, k+1) waiting likewise (see mlbm::flush_fill).
struct FillJob {
  int k;
  void* pdf_c;
  const void* cap_fine;
  void* cap_coarse;
  void* pdf_f;
};

// Adjoint state: the tape of one coarse step and the lambda arrays.
struct AdjLevel {
  std::vector<void*> X;        // tape pdf arrays, substeps 0..2^k
  const void* X0 = nullptr;    // when set, substep 0 of the tape (a checkpoint's array)
  std::vector<void*> cap;      // tape capture records, substeps 0..2^k-1
  void* lam[2] = {nullptr, nullptr};
  int cur = 0;                 // lam[cur] holds dJ/dg* of the current state
  void* lam_cap = nullptr;     // record adjoints [n_cap][stride]
  int32_t* unas[2] = {nullptr, nullptr};
  int64_t n_unas[2] = {0, 0};
  int32_t* copy_el = nullptr;
  int64_t n_copy = 0;
  void* copy_tmp = nullptr;
  int32_t* csr_ptr = nullptr;
  int32_t* csr_ent = nullptr;
  void* T = nullptr;
  // transpose of the curved-wall pre-pass (the plan's wadj_* tables)
  int64_t n_wadj = 0;
  int32_t* wadj_ent = nullptr;
  int32_t* wadj_ptr = nullptr;
  int32_t* wadj_src = nullptr;
  double* wadj_coef = nullptr;
  double* wadj_seed = nullptr;
  void* wadj_tmp = nullptr;    // [n_wadj] compute type
};

struct AdjState {
  bool attached = false;
  std::vector<AdjLevel> lv;
  double* part = nullptr;      // per-block partial records
  int64_t part_records = 0;
  AdjOp* ops_step = nullptr;   // device op lists for the reductions
  AdjOp* ops_init = nullptr;
  int n_ops_step = 0, n_ops_init = 0;
  AdjChunk* chunks_step = nullptr;  // first-stage chunks of each list
  AdjChunk* chunks_init = nullptr;
  int n_chunks_step = 0, n_chunks_init = 0;
  double* chunk_sums = nullptr;
  double* acc = nullptr;       // [nlev] d/d omega_L, then d/d u_in (3)
  // second stream for the source/ghost tail of the reverse stream-collide,
  // which runs beside the plain range (default priority, non-blocking)
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};

struct SimState {
  int stencil = 0, d = 3, q = 19, precision = 0, level0 = 0;
  int device = 0;                      // HIP device current at creation
  int n_sub = 2;                       // steps of level L+1 per step of L: 2 acoustic,
                                       // 4 diffusive scaling (Sec. 2.2)
  double tau0 = 1.0, rho0 = 1.0, u_in[3] = {0, 0, 0};
  double wr[27], geq[27];
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  std::vector<DevLevel> lv;
  uint32_t* status = nullptr;
  double* partial = nullptr;
  void* diag_levels = nullptr;
  double* maxdev = nullptr;
  void* geq_dev = nullptr;             // [q] EQ-face values in the compute type
  std::vector<bool> inited;
  bool filled = false;
  int64_t time = 0;
  Profiler prof;
  // when set, the next stream-collide launch records these events with its
  // own dispatch timestamps (start, stop)
  hipEvent_t launch_ev[2] = {nullptr, nullptr};
  std::vector<ScJob> pending;          // stream-collides not yet launched
  std::vector<FillJob> pending_fill;   // fills not yet launched
  AdjState adj;
  // graphs of two coarse steps, keyed by the parity state they start from
  hipStream_t capture_stream = nullptr;
  bool use_graphs = true;
  bool graph_fallback = false;         // capture failed; reported by mlbm_status
  std::vector<std::pair<uint64_t, hipGraphExec_t>> graphs;
  void drop_graphs();
  ~SimState();
};

struct CheckpointHeader {
  uint64_t magic;
  int64_t time;
  int32_t nlev, precision;
  int32_t f16_exp[16];
};

size_t layout_workspace(const mlbm_plan& P, int precision, char* base, SimState* s);

// Row stride of a level's [q][ld] arrays (pdfs, lambda, tape): the element
// count rounded up to 64, so that every row starts on a 128-byte line and a
// work-group's 256 consecutive elements of a row can be written with
// aligned 16-byte stores.  Entries [n, ld) of a row are never read.
inline int64_t row_stride(int64_t n) { return (n + 63) & ~(int64_t)63; }
hipEvent_t prof_event(SimState& s);

}  // namespace mlbm

struct mlbm_sim {
  mlbm::SimState s;
};
