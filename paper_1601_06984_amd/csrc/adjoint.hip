// Reverse (adjoint) of the multilevel time step and its C ABI.
//
// mlbm_adjoint_step reloads the state at the start of a coarse step into a
// tape, reruns that step forward with every stream-collide writing a fresh
// array (level k keeps 2^k + 1 arrays and 2^k capture-record buffers), and
// then applies the transposed kernels in exactly the reverse order of the
// forward schedule:
//   forward  advance(k, j): SC(k, j); [advance(k+1, 2j); advance(k+1, 2j+1);
//                            GFF(k, j); GFC(k+1, 2j+2)]
//   reverse  GFC^T(k+1); GFF^T(k); reverse(k+1, 2j+1); reverse(k+1, 2j);
//            SC^T(k, j)
// Partial sums of d/d omega_L and d/d u_in are reduced deterministically.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "adjoint_kernels.hpp"
#include "launch.hpp"
#include "plan.hpp"
#include "sim.hpp"

namespace mlbm {
namespace {

size_t al(size_t v) { return (v + 255) & ~(size_t)255; }
size_t sbytes(int p) { return p == MLBM_F64 ? 8 : (p == MLBM_F32 ? 4 : 2); }
size_t cbytes(int p) { return p == MLBM_F64 ? 8 : 4; }

int64_t blocks(int64_t n, int bs) { return (n + bs - 1) / bs; }

// ---- op lists (partial-record layout), identical to the launch order ------
struct OpBuilder {
  std::vector<AdjOp> ops;
  std::vector<AdjChunk> chunks;
  int64_t off = 0;
  void add(int64_t nb, int self, int other) {
    const int32_t c0 = (int32_t)chunks.size();
    for (int64_t b = 0; b < nb; b += REDUCE_CHUNK)
      chunks.push_back(AdjChunk{off + b, std::min<int64_t>(REDUCE_CHUNK, nb - b)});
    ops.push_back(AdjOp{off, nb, self, other, c0, (int32_t)chunks.size() - c0});
    off += nb;
  }
};

void step_ops(const SimState& s, int k, int j, OpBuilder& ob) {
  const int nlev = (int)s.lv.size();
  if (k + 1 < nlev) {
    const auto& F = s.lv[k + 1];
    if (F.n_groups) ob.add(blocks(F.n_groups, 64 / group_children(s.d)), k + 1, k);
    if (s.lv[k].n_gff) ob.add(blocks(s.lv[k].n_gff, 64), k, k + 1);
    step_ops(s, k + 1, 2 * j + 1, ob);
    step_ops(s, k + 1, 2 * j, ob);
  }
  const auto& L = s.lv[k];
  const bool first = k > 0 && (j % 2 == 0);
  const int64_t cb = (L.n_fluid - L.n_cap_fluid) / NBR_BLOCK * NBR_BLOCK;
  ob.add(blocks(cb, 256) + blocks(L.n_fluid + (first ? L.n_inner : 0) - cb, 256), k, -1);
}

void init_ops(const SimState& s, OpBuilder& ob) {
  const int nlev = (int)s.lv.size();
  for (int k = nlev - 1; k >= 1; --k)
    if (s.lv[k].n_groups) ob.add(blocks(s.lv[k].n_groups, 64 / group_children(s.d)), k, k - 1);
  for (int k = nlev - 2; k >= 0; --k)
    if (s.lv[k].n_gff) ob.add(blocks(s.lv[k].n_gff, 64), k, k + 1);
  for (int k = 0; k < nlev; ++k) ob.add(blocks(s.lv[k].n_fluid, 256), k, -1);
}

size_t layout_adjoint(const SimState& s, const mlbm_plan& P, char* base, AdjState* a,
                      const OpBuilder& os, const OpBuilder& oi) {
  size_t off = 0;
  auto take = [&](size_t b) -> char* {
    char* p = base ? base + off : nullptr;
    off += al(b);
    return p;
  };
  const int q = s.q, d = s.d;
  const size_t sb = sbytes(s.precision), cb = cbytes(s.precision);
  const size_t st = cap_stride(q);
  for (int k = 0; k < P.nlev(); ++k) {
    const auto& lp = P.lv[k];
    AdjLevel* A = a ? &a->lv[k] : nullptr;
    const int sub = 1 << k;
    for (int j = 0; j <= sub; ++j) {
      char* p = take((size_t)q * row_stride(lp.n) * sb);
      if (A) A->X[j] = p;
    }
    for (int j = 0; j < sub; ++j) {
      char* p = take((size_t)lp.n_cap() * st * cb);
      if (A) A->cap[j] = p;
    }
    char* l0 = take((size_t)q * row_stride(lp.n) * cb);
    char* l1 = take((size_t)q * row_stride(lp.n) * cb);
    char* lc = take((size_t)lp.n_cap() * st * cb);
    char* u0 = take(lp.unassigned[0].size() * 4);
    char* u1 = take(lp.unassigned[1].size() * 4);
    char* ce = take(lp.copy_elems.size() * 4);
    char* ct = take(lp.copy_elems.size() * q * cb);
    char* cp = take(lp.csr_ptr.size() * 4);
    char* cn = take(lp.csr_ent.size() * 4);
    char* T = take((size_t)group_slots(d) * lp.n_groups * st * cb);
    char* we = take(lp.wadj_ent.size() * 4);
    char* wp = take(lp.wadj_ptr.size() * 4);
    char* ws = take(lp.wadj_src.size() * 4);
    char* wc = take(lp.wadj_coef.size() * 8);
    char* wd = take(lp.wadj_seed.size() * 8);
    char* wt = take((size_t)lp.n_wadj() * cb);
    if (A) {
      A->lam[0] = l0;
      A->lam[1] = l1;
      A->lam_cap = lc;
      A->unas[0] = (int32_t*)u0;
      A->unas[1] = (int32_t*)u1;
      A->n_unas[0] = (int64_t)lp.unassigned[0].size() / 2;
      A->n_unas[1] = (int64_t)lp.unassigned[1].size() / 2;
      A->copy_el = (int32_t*)ce;
      A->n_copy = (int64_t)lp.copy_elems.size();
      A->copy_tmp = ct;
      A->csr_ptr = (int32_t*)cp;
      A->csr_ent = (int32_t*)cn;
      A->T = T;
      A->n_wadj = lp.n_wadj();
      A->wadj_ent = (int32_t*)we;
      A->wadj_ptr = (int32_t*)wp;
      A->wadj_src = (int32_t*)ws;
      A->wadj_coef = (double*)wc;
      A->wadj_seed = (double*)wd;
      A->wadj_tmp = wt;
    }
  }
  const int64_t rec = std::max(os.off, oi.off);
  char* part = take((size_t)rec * DPART * 8);
  char* ops1 = take(os.ops.size() * sizeof(AdjOp));
  char* ops2 = take(oi.ops.size() * sizeof(AdjOp));
  char* ch1 = take(os.chunks.size() * sizeof(AdjChunk));
  char* ch2 = take(oi.chunks.size() * sizeof(AdjChunk));
  char* chs = take(std::max(os.chunks.size(), oi.chunks.size()) * DPART * 8);
  char* acc = take((size_t)(P.nlev() + 3) * 8);
  if (a) {
    a->part = (double*)part;
    a->part_records = rec;
    a->ops_step = (AdjOp*)ops1;
    a->ops_init = (AdjOp*)ops2;
    a->n_ops_step = (int)os.ops.size();
    a->n_ops_init = (int)oi.ops.size();
    a->chunks_step = (AdjChunk*)ch1;
    a->chunks_init = (AdjChunk*)ch2;
    a->n_chunks_step = (int)os.chunks.size();
    a->n_chunks_init = (int)oi.chunks.size();
    a->chunk_sums = (double*)chs;
    a->acc = (double*)acc;
  }
  return off;
}

// ---- per (lattice, precision) reverse launchers -----------------------------
template <class Lat, int P>
struct Adj {
  using S = typename Prec<P>::S;
  using C = typename Prec<P>::C;
  using I = Impl<Lat, P>;

  static const void* X_of(const AdjLevel& A, int j) { return (j == 0 && A.X0) ? A.X0 : A.X[j]; }

  // forward rerun of one coarse step on the tape; as in the forward
  // schedule, consecutive stream-collides of different levels share a
  // launch (queued in `q`), and so do consecutive fills (`qf`)
  static void tape_flush(SimState& s, std::vector<ScJob>& q) {
    if (q.empty()) return;
    I::stream_collide_multi(s, q.data(), (int)q.size());
    q.clear();
  }
  static void tape_flush_fill(SimState& s, std::vector<FillJob>& qf) {
    if (qf.empty()) return;
    I::fill_sync_multi(s, qf.data(), (int)qf.size());
    qf.clear();
  }
  static void tape_advance(SimState& s, int k, int j, std::vector<ScJob>& q,
                           std::vector<FillJob>& qf) {
    AdjLevel& A = s.adj.lv[k];
    DevLevel& L = s.lv[k];
    const bool first = k > 0 && (j % 2 == 0);
    tape_flush_fill(s, qf);
    for (const auto& jb : q)
      if (jb.k == k) {
        tape_flush(s, q);
        break;
      }
    if ((int)q.size() == SC_MAX_SEG) tape_flush(s, q);
    // the last substep of the coarse step: its state X[2^k] is read by no
    // transposed kernel (each reverse stream-collide gathers from the state
    // it consumed; the fills' transposes read records), so only the
    // interpolation sources, whose records the fills use, are updated
    const bool last = j == (1 << k) - 1;
    q.push_back(ScJob{k, L.n_fluid + (first ? L.n_inner : 0), X_of(A, j), A.X[j + 1], A.cap[j],
                      last ? L.n_fluid - L.n_cap_fluid : 0});
    if (k + 1 < (int)s.lv.size()) {
      tape_advance(s, k + 1, 2 * j, q, qf);
      tape_advance(s, k + 1, 2 * j + 1, q, qf);
      tape_flush(s, q);
      if ((int)qf.size() == FILL_MAX_SEG) tape_flush_fill(s, qf);
      qf.push_back(FillJob{k, A.X[j + 1], s.adj.lv[k + 1].cap[2 * j + 1], A.cap[j],
                           s.adj.lv[k + 1].X[2 * j + 2]});
    }
  }

  static C* lam_of(SimState& s, int k, int j) {
    AdjLevel& A = s.adj.lv[k];
    const int sub = 1 << k;
    return (C*)A.lam[A.cur ^ ((sub - j) & 1)];
  }

  static void gfc_reverse(SimState& s, int k, const void* cap_coarse, C* lam, int64_t& off) {
    DevLevel& L = s.lv[k];
    AdjLevel& A = s.adj.lv[k];
    if (!L.n_groups) return;
    const DevLevel& Cl = s.lv[k - 1];
    const int64_t nb = blocks(L.n_groups, 64 / group_children(Lat::D));
    hipLaunchKernelGGL((k_adj_gfc<Lat, P>), dim3((unsigned)nb), dim3(64), 0, s.stream,
                       L.n_groups, (const int32_t*)L.grp_src, (const int32_t*)L.grp_child,
                       (const C*)cap_coarse, lam, L.ld, (C*)A.T, (C)L.omega, (C)Cl.omega,
                       (C)s.rho0, s.adj.part + off * DPART);
    off += nb;
    constexpr int W = cap_used(Lat::Q);
    const int64_t work = Cl.n_cap * W;
    hipLaunchKernelGGL((k_adj_gfc_gather<Lat, C>), dim3((unsigned)blocks(work, 256)), dim3(256), 0,
                       s.stream, A.csr_ptr, A.csr_ent, Cl.n_cap, (const C*)A.T,
                       (C*)s.adj.lv[k - 1].lam_cap);
  }

  static void gff_reverse(SimState& s, int k, const void* cap_fine, C* lam, int64_t& off) {
    DevLevel& L = s.lv[k];
    if (!L.n_gff) return;
    const DevLevel& F = s.lv[k + 1];
    const int64_t nb = blocks(L.n_gff, 64);
    hipLaunchKernelGGL((k_adj_gff<Lat, P>), dim3((unsigned)nb), dim3(64), 0, s.stream,
                       L.n_fluid + L.n_inner + L.n_outer, L.n_gff, L.gff_slot, (const C*)cap_fine,
                       (const C*)lam, L.ld, (C*)s.adj.lv[k].lam_cap, L.n_cap_fluid,
                       (C*)s.adj.lv[k + 1].lam_cap, (C)L.omega, (C)F.omega, (C)s.rho0,
                       s.adj.part + off * DPART);
    off += nb;
  }

  // One reverse stream-collide: level k, sub-step j, its tape state X and
  // its partial-record offset.
  struct RevJob {
    int k, v;
    const void* X;
    int64_t n_act, cb, nb1, nb2, off;
    C* lnew;
    C* lold;
  };

  static void rev_segment(SimState& s, const RevJob& jb, bool tail, AdjScMulti<C, S, Lat::Q>& m,
                          int64_t& total) {
    const int64_t nb = tail ? jb.nb2 : jb.nb1;
    if (!nb) return;
    auto& f = m.seg[m.nseg++];
    f.first = total;
    f.nb = nb;
    f.X = (const S*)jb.X;
    f.x0 = tail ? jb.cb : 0;
    f.x1 = tail ? jb.n_act : jb.cb;
    f.a = level_args<C, Lat::Q>(s, jb.k);
    f.lam_new = jb.lnew;
    f.lam_cap = (C*)s.adj.lv[jb.k].lam_cap;
    f.lam_old = jb.lold;
    f.part = s.adj.part + (jb.off + (tail ? jb.nb1 : 0)) * DPART;
    total += (nb + 7) / 8 * 8;
  }

  // Launches reverse stream-collides of distinct levels together: zeroing
  // and copy-link kernels per level around one tail launch (sources and
  // inner ghosts: more work per element, few blocks) on the side stream
  // beside one plain launch; all of them read lam_new and scatter to
  // disjoint lam_old entries.  A profiled run launches one level at a time
  // on one stream, timing it with events.
  static void rev_run(SimState& s, const RevJob* jobs, int n) {
    if (!n) return;
    for (int t = 0; t < n; ++t) {
      const RevJob& jb = jobs[t];
      DevLevel& L = s.lv[jb.k];
      AdjLevel& A = s.adj.lv[jb.k];
      // entries no pull assigns: the ghost rows and the listed fluid entries
      // ghost rows [n_fluid, ld) (padding included) and the listed entries
      const int64_t nz = (L.ld - L.n_fluid) * Lat::Q + A.n_unas[jb.v];
      if (nz)
        hipLaunchKernelGGL((k_zero_unassigned<C>), dim3((unsigned)blocks(nz, 256)), dim3(256), 0,
                           s.stream, jb.lold, L.ld, L.n_fluid, Lat::Q, A.unas[jb.v], A.n_unas[jb.v]);
      if (A.n_copy)
        hipLaunchKernelGGL((k_adj_copy_pre<Lat, P>), dim3((unsigned)blocks(A.n_copy, 256)), dim3(256),
                           0, s.stream, (const S*)jb.X, A.copy_el, A.n_copy, jb.n_act,
                           level_args<C, Lat::Q>(s, jb.k), (const C*)jb.lnew,
                           (const C*)A.lam_cap, (C*)A.copy_tmp);
    }
    AdjScMulti<C, S, Lat::Q> mt{}, mp{};
    int64_t nt = 0, np = 0;
    for (int t = 0; t < n; ++t) {
      rev_segment(s, jobs[t], true, mt, nt);
      rev_segment(s, jobs[t], false, mp, np);
    }
    // profiling: the first launch records the start, the last the end
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (s.prof.on && n == 1 && nt + np > 0) {
      e0 = prof_event(s);
      e1 = prof_event(s);
    }
    const bool ev = e0 && e1;
    const bool fork = nt && np && !s.prof.on && s.adj.side;
    hipStream_t tail_stream = s.stream;
    if (fork && hipEventRecord(s.adj.fork, s.stream) == hipSuccess &&
        hipStreamWaitEvent(s.adj.side, s.adj.fork, 0) == hipSuccess)
      tail_stream = s.adj.side;
    if (nt)
      launch_timed(k_adj_sc<Lat, P, true>, dim3((unsigned)nt), dim3(256), tail_stream,
                   ev ? e0 : nullptr, (ev && !np) ? e1 : nullptr, mt);
    if (np)
      launch_timed(k_adj_sc<Lat, P, false>, dim3((unsigned)np), dim3(256), s.stream,
                   (ev && !nt) ? e0 : nullptr, ev ? e1 : nullptr, mp);
    if (tail_stream != s.stream) {
      (void)hipEventRecord(s.adj.join, tail_stream);
      (void)hipStreamWaitEvent(s.stream, s.adj.join, 0);
    }
    if (ev) s.prof.rec.push_back({1, jobs[0].k, jobs[0].n_act, e0, e1});
    for (int t = 0; t < n; ++t) {
      const RevJob& jb = jobs[t];
      AdjLevel& A = s.adj.lv[jb.k];
      if (A.n_copy)
        hipLaunchKernelGGL((k_adj_copy_add<Lat::Q, C>), dim3((unsigned)blocks(A.n_copy, 256)),
                           dim3(256), 0, s.stream, A.copy_el, A.n_copy, s.lv[jb.k].ld,
                           (const C*)A.copy_tmp, jb.lold);
      // the stream-collide consumed the state after the curved-wall
      // pre-pass: carry its adjoint back through the pre-pass
      if (A.n_wadj) {
        hipLaunchKernelGGL((k_adj_wall_gather<C>), dim3((unsigned)blocks(A.n_wadj, 256)),
                           dim3(256), 0, s.stream, (const int4*)A.wadj_ent, A.wadj_ptr,
                           (const int2*)A.wadj_src, A.wadj_coef, A.n_wadj, s.lv[jb.k].ld,
                           (const C*)jb.lold, (C*)A.wadj_tmp);
        hipLaunchKernelGGL((k_adj_wall_store<C>), dim3((unsigned)blocks(A.n_wadj, 256)),
                           dim3(256), 0, s.stream, (const int4*)A.wadj_ent, A.n_wadj,
                           s.lv[jb.k].ld, (const C*)A.wadj_tmp, jb.lold);
      }
    }
  }

  static void rev_flush(SimState& s, std::vector<RevJob>& q) {
    rev_run(s, q.data(), (int)q.size());
    q.clear();
  }

  // Queues the reverse stream-collide of level k, sub-step j (partial
  // records from `off` on); consecutive ones of different levels share
  // launches.
  static void sc_reverse(SimState& s, int k, int j, const void* X, int64_t& off,
                         std::vector<RevJob>& q) {
    DevLevel& L = s.lv[k];
    const bool first = k > 0 && (j % 2 == 0);
    RevJob jb;
    jb.k = k;
    jb.v = first ? 1 : 0;
    jb.X = X;
    jb.n_act = L.n_fluid + (first ? L.n_inner : 0);
    // plain fluid [0, cb) without records; the split is rounded down to a
    // pull-table block so each work-group covers one block
    jb.cb = (L.n_fluid - L.n_cap_fluid) / NBR_BLOCK * NBR_BLOCK;
    jb.nb1 = blocks(jb.cb, 256);
    jb.nb2 = blocks(jb.n_act - jb.cb, 256);
    jb.off = off;
    jb.lnew = lam_of(s, k, j + 1);
    jb.lold = lam_of(s, k, j);
    off += jb.nb1 + jb.nb2;
    if (s.prof.on) {
      rev_flush(s, q);
      rev_run(s, &jb, 1);
      return;
    }
    for (const auto& o : q)
      if (o.k == k) {
        rev_flush(s, q);
        break;
      }
    if ((int)q.size() == ADJ_MAX_SEG) rev_flush(s, q);
    q.push_back(jb);
  }

  static void reverse(SimState& s, int k, int j, int64_t& off, std::vector<RevJob>& q) {
    const int nlev = (int)s.lv.size();
    AdjLevel& A = s.adj.lv[k];
    if (k + 1 < nlev) {
      AdjLevel& F = s.adj.lv[k + 1];
      rev_flush(s, q);   // the fill transposes read the lambdas they leave
      gfc_reverse(s, k + 1, A.cap[j], lam_of(s, k + 1, 2 * j + 2), off);
      gff_reverse(s, k, F.cap[2 * j + 1], lam_of(s, k, j + 1), off);
      reverse(s, k + 1, 2 * j + 1, off, q);
      reverse(s, k + 1, 2 * j, off, q);
    }
    sc_reverse(s, k, j, X_of(A, j), off, q);
  }

  static void seed(SimState& s, int objective) {
    for (size_t k = 0; k < s.lv.size(); ++k) {
      DevLevel& L = s.lv[k];
      AdjLevel& A = s.adj.lv[k];
      C* lam = (C*)A.lam[A.cur];
      auto a = level_args<C, Lat::Q>(s, (int)k);
      if (objective == MLBM_OBJ_KE) {
        const double vol = std::ldexp(1.0, -s.d * (int)k);
        hipLaunchKernelGGL((k_seed_ke<Lat, P>), dim3((unsigned)blocks(L.n, 256)), dim3(256), 0,
                           s.stream, (const S*)L.pdf[L.parity], a, vol, lam);
      } else {
        hipLaunchKernelGGL((k_fill_value<C>), dim3((unsigned)blocks(L.ld * Lat::Q, 256)), dim3(256), 0,
                           s.stream, lam, L.ld * Lat::Q, C(0));
        const double scale = std::ldexp(1.0, (s.d - 1) * ((int)s.lv.size() - 1 - (int)k));
        if (L.n_bounce)
          hipLaunchKernelGGL((k_seed_drag<Lat, C>), dim3((unsigned)blocks(L.n_bounce, 256)), dim3(256),
                             0, s.stream, L.bounce, L.n_bounce, L.ld, scale, lam);
        if (A.n_wadj)
          hipLaunchKernelGGL((k_seed_wall_drag<C>), dim3((unsigned)blocks(A.n_wadj, 256)),
                             dim3(256), 0, s.stream, (const int4*)A.wadj_ent, A.wadj_ptr,
                             A.wadj_seed, A.n_wadj, L.ld, scale, lam);
      }
      const int64_t ncap = L.n_cap * cap_stride(s.q);
      if (ncap)
        hipLaunchKernelGGL((k_fill_value<C>), dim3((unsigned)blocks(ncap, 256)), dim3(256), 0, s.stream,
                           (C*)A.lam_cap, ncap, C(0));
    }
    hipLaunchKernelGGL((k_fill_value<double>), dim3(1), dim3(256), 0, s.stream, s.adj.acc,
                       (int64_t)s.lv.size() + 3, 0.0);
  }

  // deterministic two-stage reduction of the block partials into acc
  static void reduce(SimState& s, const AdjOp* ops, int n_ops, const AdjChunk* chunks,
                     int n_chunks) {
    if (n_chunks)
      hipLaunchKernelGGL(k_adj_reduce_chunks, dim3((unsigned)n_chunks), dim3(256), 0, s.stream,
                         s.adj.part, chunks, s.adj.chunk_sums);
    hipLaunchKernelGGL(k_adj_reduce, dim3(1), dim3(64), 0, s.stream, s.adj.chunk_sums, ops, n_ops,
                       s.adj.acc, (int)s.lv.size());
  }

  static void step(SimState& s) {
    std::vector<ScJob> q;
    std::vector<FillJob> qf;
    tape_advance(s, 0, 0, q, qf);
    tape_flush(s, q);
    tape_flush_fill(s, qf);
    int64_t off = 0;
    std::vector<RevJob> rq;
    reverse(s, 0, 0, off, rq);
    rev_flush(s, rq);
    reduce(s, s.adj.ops_step, s.adj.n_ops_step, s.adj.chunks_step, s.adj.n_chunks_step);
    s.adj.lv[0].cur ^= 1;  // level 0 took one substep; finer levels an even count
  }

  static void init(SimState& s, const double* const* rho, const double* const* u,
                   const double* const* S_, double* const* du, double* const* drho,
                   double* const* dS) {
    const int nlev = (int)s.lv.size();
    for (int k = 0; k < nlev; ++k)
      I::init_ptr(s, k, rho[k], u[k], S_ ? S_[k] : nullptr, s.adj.lv[k].X[0], s.adj.lv[k].cap[0]);
    for (int k = 0; k + 1 < nlev; ++k)
      I::fill_gff_ptr(s, k, s.adj.lv[k].X[0], s.adj.lv[k + 1].cap[0], s.adj.lv[k].cap[0]);
    for (int k = 1; k < nlev; ++k) I::fill_gfc_ptr(s, k, s.adj.lv[k].X[0], s.adj.lv[k - 1].cap[0]);
    int64_t off = 0;
    for (int k = nlev - 1; k >= 1; --k)
      gfc_reverse(s, k, s.adj.lv[k - 1].cap[0], (C*)s.adj.lv[k].lam[s.adj.lv[k].cur], off);
    for (int k = nlev - 2; k >= 0; --k)
      gff_reverse(s, k, s.adj.lv[k + 1].cap[0], (C*)s.adj.lv[k].lam[s.adj.lv[k].cur], off);
    for (int k = 0; k < nlev; ++k) {
      DevLevel& L = s.lv[k];
      auto a = level_args<C, Lat::Q>(s, k);
      const int64_t nb = blocks(L.n_fluid, 256);
      if (nb)
      hipLaunchKernelGGL((k_adj_init<Lat, P>), dim3((unsigned)nb), dim3(256), 0, s.stream, rho[k],
                         u[k], S_ ? S_[k] : nullptr, L.n_fluid, a, L.omega,
                         (const C*)s.adj.lv[k].lam[s.adj.lv[k].cur], (C*)s.adj.lv[k].lam_cap, du[k],
                         drho ? drho[k] : nullptr, dS ? dS[k] : nullptr, s.adj.part + off * DPART);
      off += nb;
    }
    reduce(s, s.adj.ops_init, s.adj.n_ops_init, s.adj.chunks_init, s.adj.n_chunks_init);
  }

  static void get_lambda(SimState& s, int k, double* out) {
    DevLevel& L = s.lv[k];
    AdjLevel& A = s.adj.lv[k];
    hipLaunchKernelGGL((k_to_double<C>), dim3((unsigned)blocks(L.n * Lat::Q, 256)), dim3(256), 0,
                       s.stream, (const C*)A.lam[A.cur], L.n, L.ld, L.n * Lat::Q, out);
  }
};

#define MLBM_ADJ_DISPATCH_P(s, LAT, CALL)                                             \
  do {                                                                               \
    if ((s).precision == MLBM_F64) { using J = Adj<LAT, MLBM_F64>; CALL; }            \
    else if ((s).precision == MLBM_F32) { using J = Adj<LAT, MLBM_F32>; CALL; }       \
    else { using J = Adj<LAT, MLBM_F16S>; CALL; }                                     \
  } while (0)
#define MLBM_ADJ_DISPATCH(s, CALL)                                                   \
  do {                                                                               \
    if ((s).stencil == MLBM_D3Q19) MLBM_ADJ_DISPATCH_P(s, D3Q19, CALL);              \
    else if ((s).stencil == MLBM_D3Q27) MLBM_ADJ_DISPATCH_P(s, D3Q27, CALL);         \
    else MLBM_ADJ_DISPATCH_P(s, D2Q9, CALL);                                         \
  } while (0)

bool plan_matches(const SimState& s, const mlbm_plan& P) {
  if ((int)s.lv.size() != P.nlev() || s.d != P.d || s.stencil != P.stencil) return false;
  for (int k = 0; k < P.nlev(); ++k)
    if (s.lv[k].n != P.lv[k].n || s.lv[k].n_fluid != P.lv[k].n_fluid ||
        s.lv[k].n_cap != P.lv[k].n_cap())
      return false;
  return true;
}

int32_t hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(MLBM_E_HIP, "%s: %s", what, hipGetErrorString(e));
  const hipError_t l = hipGetLastError();
  if (l != hipSuccess) return fail(MLBM_E_HIP, "%s: %s", what, hipGetErrorString(l));
  return MLBM_OK;
}

}  // namespace
}  // namespace mlbm

using namespace mlbm;


extern "C" {

int32_t mlbm_adjoint_workspace_bytes(const mlbm_sim* sim, const mlbm_plan* plan, size_t* bytes) {
  if (!sim || !plan || !bytes) return fail(MLBM_E_ARG, "NULL argument");
  if (sim->s.n_sub != 2)
    return fail(MLBM_E_STATE, "the adjoint covers acoustic scaling (two fine steps per coarse "
                              "step) only");
  const SimState& s = sim->s;
  if (!plan_matches(s, *plan)) return fail(MLBM_E_ARG, "plan does not belong to this simulation");
  OpBuilder os, oi;
  step_ops(s, 0, 0, os);
  init_ops(s, oi);
  *bytes = layout_adjoint(s, *plan, nullptr, nullptr, os, oi);
  return MLBM_OK;
}

int32_t mlbm_adjoint_attach(mlbm_sim* sim, const mlbm_plan* plan, void* workspace, size_t bytes) {
  if (!sim || !plan || !workspace) return fail(MLBM_E_ARG, "NULL argument");
  SimState& s = sim->s;
  if (!plan_matches(s, *plan)) return fail(MLBM_E_ARG, "plan does not belong to this simulation");
  if (s.n_sub != 2)
    return fail(MLBM_E_STATE, "the adjoint covers acoustic scaling (two fine steps per coarse "
                              "step) only");
  if (((uintptr_t)workspace) & 255) return fail(MLBM_E_ARG, "workspace must be 256-byte aligned");
  OpBuilder os, oi;
  step_ops(s, 0, 0, os);
  init_ops(s, oi);
  const size_t need = layout_adjoint(s, *plan, nullptr, nullptr, os, oi);
  if (bytes < need) return fail(MLBM_E_ARG, "adjoint workspace too small: need %zu bytes", need);
  AdjState& a = s.adj;
  a.lv.assign(s.lv.size(), AdjLevel());
  for (size_t k = 0; k < s.lv.size(); ++k) {
    a.lv[k].X.assign(((size_t)1 << k) + 1, nullptr);
    a.lv[k].cap.assign((size_t)1 << k, nullptr);
  }
  layout_adjoint(s, *plan, (char*)workspace, &a, os, oi);
  hipError_t e = hipSuccess;
  auto up = [&](void* dst, const void* src, size_t b) {
    if (b && e == hipSuccess) e = hipMemcpyAsync(dst, src, b, hipMemcpyHostToDevice, s.stream);
  };
  for (int k = 0; k < plan->nlev(); ++k) {
    const auto& lp = plan->lv[k];
    AdjLevel& A = a.lv[k];
    up(A.unas[0], lp.unassigned[0].data(), lp.unassigned[0].size() * 4);
    up(A.unas[1], lp.unassigned[1].data(), lp.unassigned[1].size() * 4);
    up(A.copy_el, lp.copy_elems.data(), lp.copy_elems.size() * 4);
    up(A.csr_ptr, lp.csr_ptr.data(), lp.csr_ptr.size() * 4);
    up(A.csr_ent, lp.csr_ent.data(), lp.csr_ent.size() * 4);
    up(A.wadj_ent, lp.wadj_ent.data(), lp.wadj_ent.size() * 4);
    up(A.wadj_ptr, lp.wadj_ptr.data(), lp.wadj_ptr.size() * 4);
    up(A.wadj_src, lp.wadj_src.data(), lp.wadj_src.size() * 4);
    up(A.wadj_coef, lp.wadj_coef.data(), lp.wadj_coef.size() * 8);
    up(A.wadj_seed, lp.wadj_seed.data(), lp.wadj_seed.size() * 8);
    A.cur = 0;
  }
  up(a.ops_step, os.ops.data(), os.ops.size() * sizeof(AdjOp));
  up(a.ops_init, oi.ops.data(), oi.ops.size() * sizeof(AdjOp));
  up(a.chunks_step, os.chunks.data(), os.chunks.size() * sizeof(AdjChunk));
  up(a.chunks_init, oi.chunks.data(), oi.chunks.size() * sizeof(AdjChunk));
  if (e == hipSuccess) e = hipStreamSynchronize(s.stream);
  if (e != hipSuccess) return fail(MLBM_E_HIP, "adjoint attach: %s", hipGetErrorString(e));
  a.attached = true;
  return MLBM_OK;
}

int32_t mlbm_adjoint_seed(mlbm_sim* sim, int32_t objective) {
  if (!sim) return fail(MLBM_E_ARG, "sim is NULL");
  SimState& s = sim->s;
  if (!s.adj.attached) return fail(MLBM_E_STATE, "mlbm_adjoint_attach first");
  if (!s.filled) return fail(MLBM_E_STATE, "no forward state to seed from");
  if (objective != MLBM_OBJ_KE && objective != MLBM_OBJ_DRAG_X)
    return fail(MLBM_E_ARG, "unknown objective %d", objective);
  MLBM_ADJ_DISPATCH(s, J::seed(s, objective));
  return hip_check(hipSuccess, "mlbm_adjoint_seed");
}

int32_t mlbm_adjoint_step(mlbm_sim* sim, const void* dev_ckpt, size_t bytes) {
  if (!sim || !dev_ckpt) return fail(MLBM_E_ARG, "NULL argument");
  SimState& s = sim->s;
  if (!s.adj.attached) return fail(MLBM_E_STATE, "mlbm_adjoint_attach first");
  size_t need = 0;
  mlbm_checkpoint_bytes(sim, &need);
  if (bytes < need) return fail(MLBM_E_ARG, "checkpoint buffer too small");
  if (!s.adj.side) {
    hipError_t e = hipStreamCreateWithFlags(&s.adj.side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s.adj.fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s.adj.join, hipEventDisableTiming);
    if (e != hipSuccess) return fail(MLBM_E_HIP, "adjoint step: %s", hipGetErrorString(e));
  }
  // the checkpoint's per-level arrays are read in place as substep 0 of
  // the tape; a level with curved walls gets a copy, since the wall
  // pre-pass writes into the state its stream-collide consumes
  const char* p = (const char*)dev_ckpt;
  size_t off = 256;
  for (size_t k = 0; k < s.lv.size(); ++k) {
    const size_t nb = (size_t)s.q * s.lv[k].ld * sbytes(s.precision);
    if (s.lv[k].n_wall) {
      const hipError_t e = hipMemcpyAsync(s.adj.lv[k].X[0], p + off, nb,
                                          hipMemcpyDeviceToDevice, s.stream);
      if (e != hipSuccess) return fail(MLBM_E_HIP, "adjoint step: %s", hipGetErrorString(e));
    } else {
      s.adj.lv[k].X0 = p + off;
    }
    off += al(nb);
  }
  MLBM_ADJ_DISPATCH(s, J::step(s));
  for (auto& A : s.adj.lv) A.X0 = nullptr;
  return hip_check(hipSuccess, "mlbm_adjoint_step");
}

int32_t mlbm_adjoint_init(mlbm_sim* sim, const double* const* rho, const double* const* u,
                          const double* const* S, double* const* dJ_du, double* const* dJ_drho,
                          double* const* dJ_dS) {
  if (!sim || !rho || !u || !dJ_du) return fail(MLBM_E_ARG, "NULL argument");
  SimState& s = sim->s;
  if (!s.adj.attached) return fail(MLBM_E_STATE, "mlbm_adjoint_attach first");
  MLBM_ADJ_DISPATCH(s, J::init(s, rho, u, S, dJ_du, dJ_drho, dJ_dS));
  return hip_check(hipSuccess, "mlbm_adjoint_init");
}

int32_t mlbm_adjoint_params(mlbm_sim* sim, double* dJ_dtau0, double* dJ_domega, double* dJ_duin) {
  if (!sim) return fail(MLBM_E_ARG, "sim is NULL");
  SimState& s = sim->s;
  if (!s.adj.attached) return fail(MLBM_E_STATE, "mlbm_adjoint_attach first");
  std::vector<double> h(s.lv.size() + 3);
  hipError_t e = hipMemcpyAsync(h.data(), s.adj.acc, h.size() * 8, hipMemcpyDeviceToHost, s.stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s.stream);
  if (e != hipSuccess) return fail(MLBM_E_HIP, "adjoint params: %s", hipGetErrorString(e));
  // omega_L = 1/tau_L, tau_L = 1/2 + 2^(L-L0) (tau0 - 1/2)
  double t = 0;
  for (size_t k = 0; k < s.lv.size(); ++k) {
    const double w = s.lv[k].omega;
    t += h[k] * (-w * w * std::ldexp(1.0, (int)k));
    if (dJ_domega) dJ_domega[k] = h[k];
  }
  if (dJ_dtau0) *dJ_dtau0 = t;
  if (dJ_duin)
    for (int b = 0; b < 3; ++b) dJ_duin[b] = h[s.lv.size() + b];
  return MLBM_OK;
}

int32_t mlbm_adjoint_get_lambda(mlbm_sim* sim, int32_t k, double* dev_dst) {
  if (!sim || !dev_dst) return fail(MLBM_E_ARG, "NULL argument");
  SimState& s = sim->s;
  if (!s.adj.attached) return fail(MLBM_E_STATE, "mlbm_adjoint_attach first");
  if (k < 0 || k >= (int)s.lv.size()) return fail(MLBM_E_ARG, "level index out of range");
  MLBM_ADJ_DISPATCH(s, J::get_lambda(s, k, dev_dst));
  return hip_check(hipSuccess, "mlbm_adjoint_get_lambda");
}

}  // extern "C"
