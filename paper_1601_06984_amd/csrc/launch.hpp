// Per-(lattice, precision) kernel launchers shared by the forward path and
// the adjoint's tape.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "kernels.hpp"
#include "sim.hpp"

namespace mlbm {

template <class C, int Q>
inline LevelArgs<C, Q> level_args(const SimState& s, int k) {
  const DevLevel& L = s.lv[k];
  LevelArgs<C, Q> a;
  a.n = L.ld;   // row stride of the pdf arrays
  a.nbr16 = L.nbr16;
  a.nbase = L.nbase;
  a.nbr_wide = L.nbr_wide;
  a.nhdr = L.nhdr;
  a.morton = L.morton ? 1 : 0;
  a.ld16 = L.ld16;
  a.ldw = L.ldw;
  a.cap_begin = L.n_fluid - L.n_cap_fluid;
  a.n_fluid = L.n_fluid;
  a.omega = (C)L.omega;
  a.rho0 = (C)s.rho0;
  a.scale = (C)std::ldexp(1.0, L.f16_exp);
  a.inv_scale = (C)std::ldexp(1.0, -L.f16_exp);
  for (int i = 0; i < 4; ++i) a.wr[i] = C(0);
  for (int i = 0; i < Q; ++i) a.wr[stencil_wclass(s.stencil, i)] = (C)s.wr[i];
  a.geq = (const C*)s.geq_dev;
  a.wall = (const int4*)L.wall;
  a.wall_q = L.wall_q;
  a.n_wall = (int32_t)L.n_wall;
  for (int b = 0; b < 3; ++b) a.u_in[b] = s.u_in[b];
  return a;
}

// Unit conversions of the fills between levels k and k+1 (Sec. 2.2, Step 4
// and the velocity and density units): with n = n_sub fine steps per coarse
// step, g^neq is rescaled by omega_s / omega_t times dt_t / dt_s, velocity
// by (dt_t / dt_s) / (dx_t / dx_s) and the density deviation by its square.
// Acoustic scaling (n = 2) leaves velocity and density as they are.
struct FillUnits {
  double fneq_gff, us_gff, rs_gff;   // fine -> coarse (GhostFromFiner)
  double fneq_gfc, us_gfc, rs_gfc;   // coarse -> fine (GhostFromCoarser)
};
inline FillUnits fill_units(const SimState& s, int k) {
  const double wc = s.lv[k].omega, wf = s.lv[k + 1].omega, n = s.n_sub;
  FillUnits u;
  u.fneq_gff = (wf / wc) * n;
  u.us_gff = 0.5 * n;
  u.rs_gff = u.us_gff * u.us_gff;
  u.fneq_gfc = (wc / wf) / n;
  u.us_gfc = 2.0 / n;
  u.rs_gfc = u.us_gfc * u.us_gfc;
  return u;
}

// ---- per (lattice, precision) launchers ------------------------------------
template <class Lat, int P>
struct Impl {
  using S = typename Prec<P>::S;
  using C = typename Prec<P>::C;
  static constexpr int BS = 256;

  // Links with a wall fraction of level k: their values go into the state
  // `src` that the level's next stream-collide consumes (k_wall_prepass).
  static void wall_prepass(SimState& s, int k, const void* src) {
    DevLevel& L = s.lv[k];
    if (!L.n_wall) return;
    auto a = level_args<C, Lat::Q>(s, k);
    hipLaunchKernelGGL((k_wall_prepass<Lat, P>), dim3((unsigned)((L.n_wall + 255) / 256)),
                       dim3(256), 0, s.stream, (S*)const_cast<void*>(src), a);
  }

  // Explicit-array forms (also used by the adjoint's tape).
  static void stream_collide_ptr(SimState& s, int k, int64_t n_act, const void* src, void* dst,
                                 void* cap) {
    DevLevel& L = s.lv[k];
    if (n_act <= 0) return;
    auto a = level_args<C, Lat::Q>(s, k);
    // one launch; the block map balances the plain range and the tail
    // (capture sources, inner ghosts) over the XCDs
    wall_prepass(s, k, src);
    launch_timed(k_stream_collide<Lat, P, BS>, dim3((unsigned)((n_act + BS - 1) / BS)),
                 dim3(BS), s.stream, s.launch_ev[0], s.launch_ev[1], (const S*)src, (S*)dst,
                 n_act, a, (C*)cap, s.status);
  }

  // stream-collides of distinct levels (jobs) in one launch
  static void stream_collide_multi(SimState& s, const ScJob* jobs, int n) {
    if (n == 1 && jobs[0].x0 == 0) {
      stream_collide_ptr(s, jobs[0].k, jobs[0].n_act, jobs[0].src, jobs[0].dst, jobs[0].cap);
      return;
    }
    ScMulti<C, S, Lat::Q> m{};
    int64_t total = 0;
    m.nseg = 0;
    for (int j = 0; j < n; ++j) {
      if (jobs[j].n_act <= 0) continue;
      const int sg = m.nseg++;
      const int64_t b0 = std::min(jobs[j].x0, jobs[j].n_act - 1) / BS;
      const int64_t nb = (jobs[j].n_act + BS - 1) / BS - b0;
      m.first[sg] = total;
      m.b0[sg] = b0;
      m.nb[sg] = nb;
      m.n_act[sg] = jobs[j].n_act;
      m.src[sg] = (const S*)jobs[j].src;
      m.dst[sg] = (S*)jobs[j].dst;
      m.cap[sg] = (C*)jobs[j].cap;
      m.a[sg] = level_args<C, Lat::Q>(s, jobs[j].k);
      wall_prepass(s, jobs[j].k, jobs[j].src);
      total += (nb + 7) / 8 * 8;
    }
    if (!m.nseg) return;
    hipLaunchKernelGGL((k_stream_collide_multi<Lat, P, BS>), dim3((unsigned)total), dim3(BS), 0,
                       s.stream, m, s.status);
  }

  static void fill_gff_ptr(SimState& s, int k, void* pdf, const void* cap_fine, void* cap_coarse) {
    DevLevel& L = s.lv[k];
    if (!L.n_gff) return;
    auto a = level_args<C, Lat::Q>(s, k);
    const FillUnits fu = fill_units(s, k);
    const unsigned grid = (unsigned)((L.n_gff + 63) / 64);
    hipLaunchKernelGGL((k_fill_gff<Lat, P>), dim3(grid), dim3(64), 0, s.stream, (S*)pdf,
                       L.n_fluid + L.n_inner + L.n_outer, L.n_gff, L.gff_slot,
                       (const C*)cap_fine, (C*)cap_coarse, L.n_cap_fluid, a, (C)fu.fneq_gff,
                       (C)fu.us_gff, (C)fu.rs_gff, s.status);
  }

  static void fill_gfc_ptr(SimState& s, int k, void* pdf, const void* cap_coarse) {
    DevLevel& L = s.lv[k];
    if (!L.n_groups) return;
    auto a = level_args<C, Lat::Q>(s, k);
    const FillUnits fu = fill_units(s, k - 1);
    constexpr int GPB = 64 / group_children(Lat::D);
    const unsigned grid = (unsigned)((L.n_groups + GPB - 1) / GPB);
    hipLaunchKernelGGL((k_fill_gfc<Lat, P>), dim3(grid), dim3(64), 0, s.stream, (S*)pdf,
                       L.n_groups, L.grp_src, L.grp_child, (const C*)cap_coarse, a,
                       (C)fu.fneq_gfc, (C)fu.us_gfc, (C)fu.rs_gfc, s.status);
  }

  // GhostFromFiner of level k and GhostFromCoarser of level k+1 in one
  // launch; pdf_c / pdf_f are the arrays receiving the ghosts.  The same
  // kernel as grouped fills (one segment), so both give the same bits.
  static void fill_sync_ptr(SimState& s, int k, void* pdf_c, const void* cap_fine,
                            void* cap_coarse, void* pdf_f) {
    const FillJob job{k, pdf_c, cap_fine, cap_coarse, pdf_f};
    fill_sync_multi(s, &job, 1);
  }

  // fills of several level pairs (jobs) in one launch
  static void fill_sync_multi(SimState& s, const FillJob* jobs, int n) {
    constexpr int GPB = 64 / group_children(Lat::D);
    FillMulti<C, S, Lat::Q> m{};
    m.nseg = 0;
    int64_t total = 0;
    for (int j = 0; j < n; ++j) {
      const int k = jobs[j].k;
      DevLevel& L = s.lv[k];
      DevLevel& F = s.lv[k + 1];
      const int64_t nb_gff = (L.n_gff + 63) / 64;
      const int64_t nb_gfc = (F.n_groups + GPB - 1) / GPB;
      if (nb_gff + nb_gfc == 0) continue;
      auto& f = m.seg[m.nseg++];
      f.first = total;
      f.nb_gff = nb_gff;
      f.nb = nb_gff + nb_gfc;
      f.pdf_c = (S*)jobs[j].pdf_c;
      f.gff_begin = L.n_fluid + L.n_inner + L.n_outer;
      f.n_gff = L.n_gff;
      f.gff_slot = L.gff_slot;
      f.cap_fine = (const C*)jobs[j].cap_fine;
      f.cap_coarse = (C*)jobs[j].cap_coarse;
      f.cap_gff_begin = L.n_cap_fluid;
      f.ac = level_args<C, Lat::Q>(s, k);
      const FillUnits fu = fill_units(s, k);
      f.scale_gff = (C)fu.fneq_gff;
      f.us_gff = (C)fu.us_gff;
      f.rs_gff = (C)fu.rs_gff;
      f.pdf_f = (S*)jobs[j].pdf_f;
      f.n_groups = F.n_groups;
      f.grp_src = F.grp_src;
      f.grp_tab = (const int4*)F.grp_tab;
      f.grp_child = F.grp_child;
      f.af = level_args<C, Lat::Q>(s, k + 1);
      f.scale_gfc = (C)fu.fneq_gfc;
      f.us_gfc = (C)fu.us_gfc;
      f.rs_gfc = (C)fu.rs_gfc;
      total += f.nb;
    }
    if (!m.nseg) return;
    hipLaunchKernelGGL((k_fill_sync<Lat, P>), dim3((unsigned)total), dim3(64), 0, s.stream,
                       m, s.status);
  }

  static void fill_sync(SimState& s, int k) {
    DevLevel& L = s.lv[k];
    DevLevel& F = s.lv[k + 1];
    fill_sync_ptr(s, k, L.pdf[L.parity], F.cap, L.cap, F.pdf[F.parity]);
  }

  static void stream_collide(SimState& s, int k, int64_t n_act) {
    DevLevel& L = s.lv[k];
    stream_collide_ptr(s, k, n_act, L.pdf[L.parity], L.pdf[L.parity ^ 1], L.cap);
  }
  static void fill_gff(SimState& s, int k) {
    DevLevel& L = s.lv[k];
    if (k + 1 < (int)s.lv.size()) fill_gff_ptr(s, k, L.pdf[L.parity], s.lv[k + 1].cap, L.cap);
  }
  static void fill_gfc(SimState& s, int k) {
    DevLevel& L = s.lv[k];
    if (k > 0) fill_gfc_ptr(s, k, L.pdf[L.parity], s.lv[k - 1].cap);
  }

  static double init_maxdev(SimState& s, int k, const double* rho, const double* u,
                             const double* S_) {
    DevLevel& L = s.lv[k];
    if (!L.n_fluid) return 0.0;
    hipLaunchKernelGGL((k_init_maxdev<Lat>), dim3(256), dim3(256), 0, s.stream, rho, u, S_,
                       L.n_fluid, s.rho0, L.omega, s.maxdev);
    double host[256];
    if (hipMemcpyAsync(host, s.maxdev, sizeof host, hipMemcpyDeviceToHost, s.stream) != hipSuccess ||
        hipStreamSynchronize(s.stream) != hipSuccess)
      return -1.0;
    double m = 0;
    for (double v : host) m = std::max(m, v);
    return m;
  }

  static void init_ptr(SimState& s, int k, const double* rho, const double* u, const double* S_,
                       void* pdf, void* cap) {
    DevLevel& L = s.lv[k];
    auto a = level_args<C, Lat::Q>(s, k);
    if (L.n_fluid) {
      const unsigned grid = (unsigned)((L.n_fluid + 255) / 256);
      hipLaunchKernelGGL((k_init<Lat, P>), dim3(grid), dim3(256), 0, s.stream, rho, u, S_,
                         L.n_fluid, (S*)pdf, a, s.rho0, L.omega);
    }
    if (L.n > L.n_fluid && pdf == L.pdf[L.parity]) {
      // ghost entries of both arrays at rest until the first fill
      const unsigned gg = (unsigned)((L.n - L.n_fluid + 255) / 256);
      for (int b = 0; b < 2; ++b)
        hipLaunchKernelGGL((k_rest_ghosts<Lat, P>), dim3(gg), dim3(256), 0, s.stream,
                           (S*)L.pdf[b], L.n_fluid, L.n, a);
    }
    if (L.n_cap_fluid) {
      const unsigned gc = (unsigned)((L.n_cap_fluid + 255) / 256);
      hipLaunchKernelGGL((k_init_capture<Lat, P>), dim3(gc), dim3(256), 0, s.stream, rho, u, S_,
                         L.n_fluid, L.cap_elem, L.n_cap_fluid, (C*)cap, s.rho0, L.omega);
    }
  }
  static void init(SimState& s, int k, const double* rho, const double* u, const double* S_) {
    DevLevel& L = s.lv[k];
    init_ptr(s, k, rho, u, S_, L.pdf[L.parity], L.cap);
  }

  static void get_pdf(SimState& s, int k, double* out) {
    DevLevel& L = s.lv[k];
    if (!L.n) return;
    auto a = level_args<C, Lat::Q>(s, k);
    hipLaunchKernelGGL((k_get_pdf<Lat, P>), dim3((unsigned)((L.n + 255) / 256)), dim3(256), 0,
                       s.stream, (const S*)L.pdf[L.parity], L.n, a, out);
  }
  static void get_prev(SimState& s, int k, double* out) {
    DevLevel& L = s.lv[k];
    if (!L.n) return;
    auto a = level_args<C, Lat::Q>(s, k);
    hipLaunchKernelGGL((k_get_pdf<Lat, P>), dim3((unsigned)((L.n + 255) / 256)), dim3(256), 0,
                       s.stream, (const S*)L.pdf[L.parity ^ 1], L.n, a, out);
  }
  static void set_pdf(SimState& s, int k, const double* in) {
    DevLevel& L = s.lv[k];
    if (!L.n) return;
    auto a = level_args<C, Lat::Q>(s, k);
    hipLaunchKernelGGL((k_set_pdf<Lat, P>), dim3((unsigned)((L.n + 255) / 256)), dim3(256), 0,
                       s.stream, (S*)L.pdf[L.parity], L.n, a, in);
  }
  // pre-collision pdfs (what 0) or strain rate (what 1) of the fluid
  // elements, pulled again from the array the last stream-collide read
  static void get_pulled(SimState& s, int k, int what, double* out) {
    DevLevel& L = s.lv[k];
    if (!L.n_fluid) return;
    auto a = level_args<C, Lat::Q>(s, k);
    const dim3 grid((unsigned)((L.n_fluid + 255) / 256));
    const S* prev = (const S*)L.pdf[L.parity ^ 1];
    if (what == 0)
      hipLaunchKernelGGL((k_get_pulled<Lat, P, 0>), grid, dim3(256), 0, s.stream, prev,
                         L.n_fluid, a, L.omega, out);
    else
      hipLaunchKernelGGL((k_get_pulled<Lat, P, 1>), grid, dim3(256), 0, s.stream, prev,
                         L.n_fluid, a, L.omega, out);
  }
  static void set_pre(SimState& s, int k, const double* in) {
    DevLevel& L = s.lv[k];
    if (!L.n_fluid) return;
    auto a = level_args<C, Lat::Q>(s, k);
    hipLaunchKernelGGL((k_set_pre<Lat, P>), dim3((unsigned)((L.n_fluid + 255) / 256)), dim3(256),
                       0, s.stream, (S*)L.pdf[L.parity], L.n_fluid, a, in, (C*)L.cap, s.status);
  }
  static void get_moments(SimState& s, int k, double* out) {
    DevLevel& L = s.lv[k];
    if (!L.n_fluid) return;
    auto a = level_args<C, Lat::Q>(s, k);
    hipLaunchKernelGGL((k_get_moments<Lat, P>), dim3((unsigned)((L.n_fluid + 255) / 256)),
                       dim3(256), 0, s.stream, (const S*)L.pdf[L.parity], L.n_fluid, a, out);
  }
  static void diag_partial(SimState& s, int k) {
    diag_partial_to(s, k, s.partial + (int64_t)k * DIAG_BLOCKS * DIAG_VALS);
  }
  // level k's block partials into `partial` (DIAG_BLOCKS * DIAG_VALS doubles)
  static void diag_partial_to(SimState& s, int k, double* partial) {
    DevLevel& L = s.lv[k];
    auto a = level_args<C, Lat::Q>(s, k);
    hipLaunchKernelGGL((k_diag_partial<Lat, P>), dim3(DIAG_BLOCKS), dim3(256), 0, s.stream,
                       (const S*)L.pdf[L.parity], L.n_fluid, L.bounce, L.n_bounce, a, partial);
  }
};

// ---- dispatch -------------------------------------------------------------
#define MLBM_DISPATCH_P(s, LAT, CALL)                                       \
  do {                                                                      \
    if ((s).precision == MLBM_F64) { using I = Impl<LAT, MLBM_F64>; CALL; }  \
    else if ((s).precision == MLBM_F32) { using I = Impl<LAT, MLBM_F32>; CALL; } \
    else { using I = Impl<LAT, MLBM_F16S>; CALL; }                          \
  } while (0)
#define MLBM_DISPATCH(s, CALL)                                              \
  do {                                                                      \
    if ((s).stencil == MLBM_D3Q19) MLBM_DISPATCH_P(s, D3Q19, CALL);         \
    else if ((s).stencil == MLBM_D3Q27) MLBM_DISPATCH_P(s, D3Q27, CALL);    \
    else MLBM_DISPATCH_P(s, D2Q9, CALL);                                    \
  } while (0)


}  // namespace mlbm
