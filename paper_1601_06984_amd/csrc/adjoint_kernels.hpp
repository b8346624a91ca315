// Hand-written adjoint kernels of one multilevel time step: the transposed
// BGK collision and capture record, the pull streaming as a scatter (each
// (element, direction) entry is read by at most one pull, so the scatter is
// race-free), and the transposes of both compact-interpolation fills.
//
// Conventions: lambda arrays hold dJ/dg for the g-form pdfs, in the compute
// precision of the simulation; the storage codec is treated as identity.
// Every kernel that touches a relaxation rate adds its FP64 partials per
// block to `part` (DPART doubles per block): d/d omega of the kernel's own
// level, d/d omega of the other level it couples to, and d/d u_in.
#pragma once

#include "kernels.hpp"

namespace mlbm {

constexpr int DPART = 5;

__device__ __forceinline__ void block_sums(double* sm, const double* v, int nv, double* out) {
  // butterfly within each wavefront, then the wavefronts' sums in order:
  // a fixed sequence of additions, so the result does not depend on timing
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int k = 0; k < nv; ++k) {
    double x = v[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    if (lane == 0) sm[wave * nv + k] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 0; k < nv; ++k) {
      double t = 0;
      for (int w = 0; w < nw; ++w) t += sm[w * nv + k];
      out[k] = t;
    }
  __syncthreads();
}

// d g_eq / d(drho, rho, u) transposed: adds the contributions of lgeq.
template <class Lat, class C>
__device__ __forceinline__ void geq_adjoint(const C* lgeq, C rho, const C* u, C uu, C& ldrho,
                                            C& lrho, C* lu) {
#pragma unroll
  for (int i = 0; i < Lat::Q; ++i) {
    C cu = 0;
#pragma unroll
    for (int a = 0; a < Lat::D; ++a) cu += C(Lat::c(i, a)) * u[a];
    const C w = (C)Lat::w(i);
    const C P = C(3) * cu + C(4.5) * cu * cu - C(1.5) * uu;
    const C wl = w * lgeq[i];
    ldrho += wl;
    lrho += wl * P;
#pragma unroll
    for (int a = 0; a < Lat::D; ++a)
      lu[a] += wl * rho * (C(3) * C(Lat::c(i, a)) + C(9) * cu * C(Lat::c(i, a)) - C(3) * u[a]);
  }
}

// mu = (d g*/d g)^T lam_star + (d rec/d g)^T lam_rec for one element with
// pre-collision g; rec is the capture record (drho, u, S, g^neq).
template <class Lat, class C>
__device__ __forceinline__ void collide_adjoint(const C* g, const C* ls, const C* lrec, C rho0,
                                                C omega, C* mu, double& d_omega) {
  constexpr int D = Lat::D, Q = Lat::Q;
  C drho, rho, u[3];
  macro_g<Lat, C>(g, rho0, drho, rho, u);
  const C uu = dot_uu<Lat, C>(u);
  C geq[Q], lg[Q], lgeq[Q];
  double dw = 0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    geq[i] = geq_i<Lat, C>(i, drho, rho, u, uu);
    lg[i] = (C(1) - omega) * ls[i];
    lgeq[i] = omega * ls[i];
    dw += (double)ls[i] * (double)(geq[i] - g[i]);
  }
  C ldrho = 0, lrho = 0, lu[3] = {0, 0, 0};
  if (lrec) {
    const C pref = -C(1.5) * omega / rho;
    C S[Lat::NS];
#pragma unroll
    for (int k = 0; k < Lat::NS; ++k) {
      C pi = 0;
#pragma unroll
      for (int i = 0; i < Q; ++i) pi += C(Lat::c(i, strain_a(D, k)) * Lat::c(i, strain_b(D, k))) * (g[i] - geq[i]);
      S[k] = pref * pi;
      const C lS = lrec[cap_s(Lat::Q) + k];
      lrho -= lS * S[k] / rho;
      dw += (double)lS * (double)S[k] / (double)omega;
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      C lf = lrec[cap_fneq(Lat::Q) + i];
#pragma unroll
      for (int k = 0; k < Lat::NS; ++k)
        lf += pref * C(Lat::c(i, strain_a(D, k)) * Lat::c(i, strain_b(D, k))) * lrec[cap_s(Lat::Q) + k];
      lg[i] += lf;
      lgeq[i] -= lf;
    }
    ldrho += lrec[cap_rho(Lat::Q)];
#pragma unroll
    for (int a = 0; a < D; ++a) lu[a] += lrec[cap_u(Lat::Q) + a];
  }
  geq_adjoint<Lat, C>(lgeq, rho, u, uu, ldrho, lrho, lu);
  C lj[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < D; ++a) {
    lj[a] = lu[a] / rho;
    lrho -= lu[a] * u[a] / rho;
  }
  ldrho += lrho;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    C v = lg[i] + ldrho;
#pragma unroll
    for (int a = 0; a < D; ++a) v += C(Lat::c(i, a)) * lj[a];
    mu[i] = v;
  }
  d_omega += dw;
}

// ---------------------------------------------------------------- seeds ----
// Kinetic energy E = 1/2 V sum rho |u|^2 of the post-collision state:
// dE/dg*_i = V (c_i . u - u.u/2) on fluid elements, zero elsewhere.
template <class Lat, int P>
__global__ __launch_bounds__(256) void k_seed_ke(const typename Prec<P>::S* __restrict__ pdf,
                                                 const LevelArgs<typename Prec<P>::C, Lat::Q> a,
                                                 double vol, typename Prec<P>::C* __restrict__ lam) {
  using C = typename Prec<P>::C;
  const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (x >= a.n) return;
  if (x >= a.n_fluid) {
#pragma unroll
    for (int i = 0; i < Lat::Q; ++i) lam[(int64_t)i * a.n + x] = C(0);
    return;
  }
  C g[Lat::Q];
#pragma unroll
  for (int i = 0; i < Lat::Q; ++i) g[i] = load_g<P>(pdf, (int64_t)i * a.n + x, a.wr[Lat::wclass(i)], a.inv_scale);
  C drho, rho, u[3];
  macro_g<Lat, C>(g, a.rho0, drho, rho, u);
  const C uu = dot_uu<Lat, C>(u);
#pragma unroll
  for (int i = 0; i < Lat::Q; ++i) {
    C cu = 0;
#pragma unroll
    for (int b = 0; b < Lat::D; ++b) cu += C(Lat::c(i, b)) * u[b];
    lam[(int64_t)i * a.n + x] = (C)vol * (cu - C(0.5) * uu);
  }
}

template <class C>
__global__ __launch_bounds__(256) void k_fill_value(C* __restrict__ p, int64_t n, C v) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t < n) p[t] = v;
}

// Drag along x: d/dg*_i of sum over links 2 c_i f*_i scaled to finest units.
template <class Lat, class C>
__global__ __launch_bounds__(256) void k_seed_drag(const int32_t* __restrict__ bounce,
                                                   int64_t n_bounce, int64_t n, double scale,
                                                   C* __restrict__ lam) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= n_bounce) return;
  const int64_t x = bounce[t];
  const int i = Lat::opp(bounce[n_bounce + t]);
  lam[(int64_t)i * n + x] = (C)(2.0 * Lat::c(i, 0) * scale);
}

// Transpose of the curved-wall pre-pass (k_wall_prepass), in gather form:
// every entry e the pre-pass reads or writes gets [e not written] lam[e] +
// sum over its terms of coefficient * lam[written entry of the term's link],
// formed for all entries before any is stored (two launches), so the sums
// are fixed-order and free of races.
template <class C>
__global__ __launch_bounds__(256) void k_adj_wall_gather(
    const int4* __restrict__ ent, const int32_t* __restrict__ ptr, const int2* __restrict__ src,
    const double* __restrict__ coef, int64_t n_ent, int64_t n, const C* __restrict__ lam,
    C* __restrict__ tmp) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n_ent) return;
  const int4 r = ent[e];
  C acc = r.z ? lam[(int64_t)r.x * n + r.y] : C(0);
  for (int32_t k = ptr[e]; k < ptr[e + 1]; ++k) {
    const int2 w = src[k];
    acc += (C)coef[k] * lam[(int64_t)w.x * n + w.y];
  }
  tmp[e] = acc;
}

template <class C>
__global__ __launch_bounds__(256) void k_adj_wall_store(const int4* __restrict__ ent,
                                                        int64_t n_ent, int64_t n,
                                                        const C* __restrict__ tmp,
                                                        C* __restrict__ lam) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n_ent) return;
  const int4 r = ent[e];
  lam[(int64_t)r.x * n + r.y] = tmp[e];
}

// Drag along x with curved walls: the returning value of a link is the
// interpolated one, so d/dg* of c_ox (g*_o(x) + value) adds, over the
// entries the value reads, c_ox (coefficient - [own entry]) to the halfway
// seed 2 c_ox (k_seed_drag).
template <class C>
__global__ __launch_bounds__(256) void k_seed_wall_drag(const int4* __restrict__ ent,
                                                        const int32_t* __restrict__ ptr,
                                                        const double* __restrict__ seed,
                                                        int64_t n_ent, int64_t n, double scale,
                                                        C* __restrict__ lam) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n_ent) return;
  const int4 r = ent[e];
  double acc = 0;
  for (int32_t k = ptr[e]; k < ptr[e + 1]; ++k) acc += seed[k];
  lam[(int64_t)r.x * n + r.y] += (C)(acc * scale);
}

// ------------------------------------------------- stream-collide reverse --
// Gathers the tape state, forms mu = (d g*/d g)^T lam* [+ (d rec/d g)^T
// lam_rec] in streamed passes over the directions (no per-direction
// temporaries beyond g and lam*), and scatters each mu_i to the entry its
// pull read, with the sources decoded once for both.  COPY links are added
// by k_adj_copy_* around this kernel.  REC instantiations cover the tail
// of the element range, where capture sources (with a record adjoint) and
// inner ghosts live; the plain instantiation carries no record code and
// fits 4 waves per SIMD without spills.
// Work-group `bid` of the range [x0, x1): every thread calls it.
template <class Lat, int P, bool REC>
__device__ __forceinline__ void adj_sc_body(
    int64_t bid, const typename Prec<P>::S* __restrict__ X, int64_t x0, int64_t x1,
    const LevelArgs<typename Prec<P>::C, Lat::Q>& a,
    const typename Prec<P>::C* __restrict__ lam_new, typename Prec<P>::C* __restrict__ lam_cap,
    typename Prec<P>::C* __restrict__ lam_old, double* __restrict__ part, double* sm,
    int32_t* slots) {
  using C = typename Prec<P>::C;
  constexpr int Q = Lat::Q, D = Lat::D, NS = Lat::NS;
  // x0 is a multiple of the pull-table block: a work-group is one block,
  // holding at least one element of [x0, x1)
  const int64_t blk = (x0 >> 8) + bid;
  const int64_t x = x0 + bid * 256 + threadIdx.x;
  double acc[DPART] = {0, 0, 0, 0, 0};
  int32_t j[Q];   // pull sources: gathered from, then scattered to
  pull_sources_wg<Lat>(a, blk, (uint32_t)(x < x1 ? x : x1 - 1), j, slots);
  if (x < x1) {
    C g[Q], ls[Q];
    gather_from<Lat, P>(X, x, a, j, g);
#pragma unroll
    for (int i = 0; i < Q; ++i) ls[i] = load_elem(lam_new + (int64_t)i * a.n, a.n, (uint32_t)x);
    C drho, rho, u[3];
    macro_g<Lat, C>(g, a.rho0, drho, rho, u);
    const C uu = dot_uu<Lat, C>(u);
    const C om = a.omega;
    C ldrho = 0, lrho = 0, lu[3] = {0, 0, 0};
    double dw = 0;
    // record adjoint (capture sources only)
    C lr_S[NS], lr_f[Q], pref = 0;
    bool src = false;
    if constexpr (REC) {
      src = x >= a.cap_begin && x < a.n_fluid;
      if (src) {
        C* r = lam_cap + (x - a.cap_begin) * cap_stride(Lat::Q);
        ldrho += r[cap_rho(Lat::Q)];
#pragma unroll
        for (int b = 0; b < D; ++b) lu[b] += r[cap_u(Lat::Q) + b];
#pragma unroll
        for (int k = 0; k < NS; ++k) lr_S[k] = r[cap_s(Lat::Q) + k];
#pragma unroll
        for (int i = 0; i < Q; ++i) lr_f[i] = r[cap_fneq(Lat::Q) + i];
#pragma unroll
        for (int c = 0; c < cap_used(Lat::Q); ++c) r[c] = C(0);  // consumed
        pref = -C(1.5) * om / rho;
        // S of the record: lrho and omega contributions
        C pi[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) pi[k] = 0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          const C fneq = g[i] - geq_i<Lat, C>(i, drho, rho, u, uu);
#pragma unroll
          for (int k = 0; k < NS; ++k) {
            const int cc = Lat::c(i, strain_a(D, k)) * Lat::c(i, strain_b(D, k));
            if (cc > 0) pi[k] += fneq;
            if (cc < 0) pi[k] -= fneq;
          }
        }
#pragma unroll
        for (int k = 0; k < NS; ++k) {
          const C Sk = pref * pi[k];
          lrho -= lr_S[k] * Sk / rho;
          dw += (double)lr_S[k] * (double)Sk / (double)om;
        }
      }
    }
    auto lf_of = [&](int i) -> C {   // adjoint of g^neq_i through the record
      C lf = 0;
      if constexpr (REC) {
        if (src) {
          lf = lr_f[i];
#pragma unroll
          for (int k = 0; k < NS; ++k) {
            const int cc = Lat::c(i, strain_a(D, k)) * Lat::c(i, strain_b(D, k));
            if (cc > 0) lf += pref * lr_S[k];
            if (cc < 0) lf -= pref * lr_S[k];
          }
        }
      }
      return lf;
    };
    // pass 1: lambda of g^eq, pulled back to (drho, rho, u)
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      C cu = 0;
#pragma unroll
      for (int b = 0; b < D; ++b) {
        const int ci = Lat::c(i, b);
        if (ci > 0) cu += u[b];
        if (ci < 0) cu -= u[b];
      }
      const C w = (C)Lat::w(i);
      const C Pq = C(3) * cu + C(4.5) * cu * cu - C(1.5) * uu;
      const C geq = w * (drho + rho * Pq);
      dw += (double)ls[i] * (double)(geq - g[i]);
      const C wl = w * (om * ls[i] - lf_of(i));
      ldrho += wl;
      lrho += wl * Pq;
#pragma unroll
      for (int b = 0; b < D; ++b)
        lu[b] += wl * rho * (C(3) * C(Lat::c(i, b)) + C(9) * cu * C(Lat::c(i, b)) - C(3) * u[b]);
    }
    C lj[3] = {0, 0, 0};
#pragma unroll
    for (int b = 0; b < D; ++b) {
      lj[b] = lu[b] / rho;
      lrho -= lu[b] * u[b] / rho;
    }
    ldrho += lrho;
    // pass 2: mu_i, scattered as formed
    const C om1 = C(1) - om;
    store_elem(lam_old, a.n, (uint32_t)x, om1 * ls[0] + lf_of(0) + ldrho);
    const uint32_t nn = (uint32_t)a.n, xo = (uint32_t)x;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      C mu = om1 * ls[i] + lf_of(i) + ldrho;
#pragma unroll
      for (int b = 0; b < D; ++b) {
        const int ci = Lat::c(i, b);
        if (ci > 0) mu += lj[b];
        if (ci < 0) mu -= lj[b];
      }
      const int32_t v = j[i];
      // scatter to the entry the pull read: (i, v), or (opp(i), x) for
      // bounce-back; one descriptor over the pair of opposite rows
      const int pair = (i & 1) ? i : i - 1;
      const uint32_t off = v >= 0 ? (uint32_t)(i - pair) * nn + (uint32_t)v
                                  : (uint32_t)(Lat::opp(i) - pair) * nn + xo;
      if (v >= 0 || v == MLBM_NBR_BOUNCE) {
        store_elem(lam_old + (int64_t)pair * a.n, 2 * a.n, off, mu);
      } else if (v == MLBM_NBR_EQ) {
        // f_i = f^eq_i(rho0, u_in): d/du_in = w rho0 (3 c + 9 (c.u_in) c - 3 u_in)
        const double w = Lat::w(i);
        double cu = 0;
#pragma unroll
        for (int b = 0; b < D; ++b) cu += Lat::c(i, b) * a.u_in[b];
#pragma unroll
        for (int b = 0; b < D; ++b)
          acc[2 + b] += (double)mu * w * (double)a.rho0 *
                        (3.0 * Lat::c(i, b) + 9.0 * cu * Lat::c(i, b) - 3.0 * a.u_in[b]);
      }
    }
    acc[0] = dw;
  }
  block_sums(sm, acc, DPART, part + bid * DPART);
}

// Reverse stream-collides of several levels (segments) in one launch: the
// transposes of consecutive stream-collides of different levels touch
// disjoint data.  A single one is a launch with one segment.
constexpr int ADJ_MAX_SEG = 4;
template <class C, class S, int Q>
struct AdjScSeg {
  int64_t first, nb;   // work-groups [first, first + nb)
  const S* X;
  int64_t x0, x1;
  LevelArgs<C, Q> a;
  const C* lam_new;
  C* lam_cap;
  C* lam_old;
  double* part;
};
template <class C, class S, int Q>
struct AdjScMulti {
  int nseg;
  AdjScSeg<C, S, Q> seg[ADJ_MAX_SEG];
};

// Every segment starts at a multiple of 8 work-groups (on XCD 0), so its
// work-groups map to logical blocks by the XCD-sliced order (xcd_block):
// each XCD gathers from and scatters to one contiguous slice, whose lines
// its own L2 holds; the few work-groups between segments exit.
template <class Lat, int P, bool REC>
__global__ __launch_bounds__(256, (P != MLBM_F64 && !REC) ? 4 : 1) void k_adj_sc(
    const AdjScMulti<typename Prec<P>::C, typename Prec<P>::S, Lat::Q> m) {
  __shared__ double sm[4 * DPART];
  __shared__ int32_t slots[NBR_SLOTS];
  int sg = 0;
  while (sg + 1 < m.nseg && (int64_t)blockIdx.x >= m.seg[sg + 1].first) ++sg;
  const auto& f = m.seg[sg];
  const int64_t b = (int64_t)blockIdx.x - f.first;
  if (b >= f.nb) return;
  adj_sc_body<Lat, P, REC>(xcd_block(b, f.nb), f.X, f.x0, f.x1, f.a, f.lam_new, f.lam_cap,
                           f.lam_old, f.part, sm, slots);
}

// COPY links, part 1 (before k_adj_sc consumes the record adjoints):
// tmp[t][i] = mu_i(x) for the copied directions of element x = elems[t].
template <class Lat, int P>
__global__ __launch_bounds__(256) void k_adj_copy_pre(
    const typename Prec<P>::S* __restrict__ X, const int32_t* __restrict__ elems, int64_t n_el, int64_t n_act,
    const LevelArgs<typename Prec<P>::C, Lat::Q> a, const typename Prec<P>::C* __restrict__ lam_new,
    const typename Prec<P>::C* __restrict__ lam_cap, typename Prec<P>::C* __restrict__ tmp) {
  using C = typename Prec<P>::C;
  constexpr int Q = Lat::Q, D = Lat::D;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= n_el) return;
  const int64_t x = elems[t];
  if (x >= n_act) {
#pragma unroll
    for (int i = 0; i < Q; ++i) tmp[t * Q + i] = C(0);
    return;
  }
  C g[Q], ls[Q], mu[Q];
  gather_g<Lat, P>(X, x >> 8, x, a, g);
#pragma unroll
  for (int i = 0; i < Q; ++i) ls[i] = lam_new[(int64_t)i * a.n + x];
  const bool src = x >= a.cap_begin && x < a.n_fluid;
  double dummy = 0;
  collide_adjoint<Lat, C>(g, ls, src ? lam_cap + (x - a.cap_begin) * cap_stride(Lat::Q) : nullptr,
                          a.rho0, a.omega, mu, dummy);
  tmp[t * Q] = C(0);
#pragma unroll
  for (int i = 1; i < Q; ++i)
    tmp[t * Q + i] = pull_source<Lat>(a, x >> 8, (uint32_t)x, i) == MLBM_NBR_COPY ? mu[i] : C(0);
}

// COPY links, part 2 (after k_adj_sc): lam_old[i][x] += tmp[t][i].
template <int Q, class C>
__global__ __launch_bounds__(256) void k_adj_copy_add(const int32_t* __restrict__ elems,
                                                      int64_t n_el, int64_t n,
                                                      const C* __restrict__ tmp,
                                                      C* __restrict__ lam_old) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= n_el) return;
  const int64_t x = elems[t];
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const C v = tmp[t * Q + i];
    if (v != C(0)) lam_old[(int64_t)i * n + x] += v;
  }
}

// Both zeroings of the entries no pull assigns, in one launch: threads
// [0, (n - begin) q) clear the ghost rows, the next cnt the listed
// (element, direction) entries of the fluid range.
template <class C>
__global__ __launch_bounds__(256) void k_zero_unassigned(C* __restrict__ lam, int64_t n,
                                                         int64_t begin, int q,
                                                         const int32_t* __restrict__ list,
                                                         int64_t cnt) {
  const int64_t w = n - begin, nr = w * q;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t < nr) {
    lam[(t / w) * n + begin + t % w] = C(0);
  } else if (t - nr < cnt) {
    const int64_t e = t - nr;
    lam[(int64_t)list[cnt + e] * n + list[e]] = C(0);
  }
}

// --------------------------------------------- interpolation transposes ----
// Adjoint of the strain-rate part of the closed-form velocity: given the
// velocity adjoint lu, adds d/dS of the four sources to lS[4][NS].
// wd, wc: weights of the diagonal and (3D) cross coefficients in
// u -= wd (a_xx + a_yy + a_zz) + wc (s_x s_y a_xy + s_y s_z a_yz + s_x s_z a_xz).
template <int D, class C>
__device__ __forceinline__ void strain_terms_adjoint(const C* lu, int sx, int sy, int sz, C wd,
                                                     C wc, C (*lS)[6]) {
  if constexpr (D == 3) {
    const C sxy = C(sx * sy), syz = C(sy * sz), sxz = C(sx * sz);
    C laxx = -wd * lu[0], layy = -wd * lu[0], lazz = -wd * lu[0];
    C laxy = -wc * sxy * lu[0], layz = -wc * syz * lu[0], laxz = -wc * sxz * lu[0];
    C lbxx = -wd * lu[1], lbyy = -wd * lu[1], lbzz = -wd * lu[1];
    C lbxy = -wc * sxy * lu[1], lbyz = -wc * syz * lu[1], lbxz = -wc * sxz * lu[1];
    C lcxx = -wd * lu[2], lcyy = -wd * lu[2], lczz = -wd * lu[2];
    C lcxy = -wc * sxy * lu[2], lcyz = -wc * syz * lu[2], lcxz = -wc * sxz * lu[2];
    C lDx[6] = {0, 0, 0, 0, 0, 0}, lDy[6] = {0, 0, 0, 0, 0, 0}, lDz[6] = {0, 0, 0, 0, 0, 0};
    // a_yz = T - 2 Dx(yz), b_xz = T - 2 Dy(xz), c_xy = T - 2 Dz(xy),
    // T = Dz(xy) + Dx(yz) + Dy(xz)
    const C lT = layz + lbxz + lcxy;
    lDx[4] += lT - C(2) * layz;
    lDy[5] += lT - C(2) * lbxz;
    lDz[3] += lT - C(2) * lcxy;
    lDz[5] += lazz; lcxz -= C(0.5) * lazz;   // a_zz = Dz(xz) - c_xz/2
    lDx[5] += lcxx; laxz -= C(0.5) * lcxx;   // c_xx = Dx(xz) - a_xz/2
    lDz[4] += lbzz; lcyz -= C(0.5) * lbzz;   // b_zz = Dz(yz) - c_yz/2
    lDy[4] += lcyy; lbyz -= C(0.5) * lcyy;   // c_yy = Dy(yz) - b_yz/2
    lDy[3] += layy; lbxy -= C(0.5) * layy;   // a_yy = Dy(xy) - b_xy/2
    lDx[3] += lbxx; laxy -= C(0.5) * lbxx;   // b_xx = Dx(xy) - a_xy/2
    lDx[0] += C(0.5) * laxx; lDy[0] += laxy; lDz[0] += laxz;
    lDx[1] += lbxy; lDy[1] += C(0.5) * lbyy; lDz[1] += lbyz;
    lDx[2] += lcxz; lDy[2] += lcyz; lDz[2] += C(0.5) * lczz;
    const C hx = C(0.5) * sx, hy = C(0.5) * sy, hz = C(0.5) * sz;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const C ex = hx * lDx[c], ey = hy * lDy[c], ez = hz * lDz[c];
      lS[0][c] += -ex - ey - ez;   // H
      lS[1][c] += ex + ey - ez;    // K
      lS[2][c] += ex - ey + ez;    // M
      lS[3][c] += -ex + ey + ez;   // N
    }
  } else {
    (void)sz;
    (void)wc;
    const C laxx = -wd * lu[0], layy = -wd * lu[0];
    const C lbxx = -wd * lu[1], lbyy = -wd * lu[1];
    C lDx[3] = {0, 0, 0}, lDy[3] = {0, 0, 0};
    lDx[2] += lbxx;                     // b_xx = Dx(xy) - a_xy/2
    const C laxy = -C(0.5) * lbxx;
    lDy[2] += layy;                     // a_yy = Dy(xy) - b_xy/2
    const C lbxy = -C(0.5) * layy;
    lDx[0] += C(0.5) * laxx;
    lDy[0] += laxy;
    lDx[1] += lbxy;
    lDy[1] += C(0.5) * lbyy;
    const C hx = C(0.5) * sx, hy = C(0.5) * sy;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const C ex = hx * lDx[c], ey = hy * lDy[c];
      lS[0][c] += -ex - ey;   // P
      lS[1][c] += ex - ey;    // P + s_x
      lS[2][c] += -ex + ey;   // P + s_y
      lS[3][c] += ex + ey;    // P + s_x + s_y
    }
  }
}

// Forward closed form of the strain part (same as the fill kernels), used to
// recompute the interpolated velocity in the reverse kernels.
template <int D, class C>
__device__ __forceinline__ void strain_terms(const C* const* S, int sx, int sy, int sz, C wd, C wc,
                                             C* u) {
  if constexpr (D == 3) {
    const C hx = C(0.5) * sx, hy = C(0.5) * sy, hz = C(0.5) * sz;
    auto Dx = [&](int k) { return hx * (-S[0][k] + S[1][k] + S[2][k] - S[3][k]); };
    auto Dy = [&](int k) { return hy * (-S[0][k] + S[1][k] - S[2][k] + S[3][k]); };
    auto Dz = [&](int k) { return hz * (-S[0][k] - S[1][k] + S[2][k] + S[3][k]); };
    const C axx = C(0.5) * Dx(0), axy = Dy(0), axz = Dz(0);
    const C bxy = Dx(1), byy = C(0.5) * Dy(1), byz = Dz(1);
    const C cxz = Dx(2), cyz = Dy(2), czz = C(0.5) * Dz(2);
    const C bxx = Dx(3) - C(0.5) * axy, ayy = Dy(3) - C(0.5) * bxy;
    const C cyy = Dy(4) - C(0.5) * byz, bzz = Dz(4) - C(0.5) * cyz;
    const C cxx = Dx(5) - C(0.5) * axz, azz = Dz(5) - C(0.5) * cxz;
    const C T = Dz(3) + Dx(4) + Dy(5);
    const C ayz = T - C(2) * Dx(4), bxz = T - C(2) * Dy(5), cxy = T - C(2) * Dz(3);
    const C sxy = C(sx * sy), syz = C(sy * sz), sxz = C(sx * sz);
    u[0] -= wd * (axx + ayy + azz) + wc * (sxy * axy + syz * ayz + sxz * axz);
    u[1] -= wd * (bxx + byy + bzz) + wc * (sxy * bxy + syz * byz + sxz * bxz);
    u[2] -= wd * (cxx + cyy + czz) + wc * (sxy * cxy + syz * cyz + sxz * cxz);
  } else {
    (void)sz;
    (void)wc;
    const C hx = C(0.5) * sx, hy = C(0.5) * sy;
    auto Dx = [&](int k) { return hx * (-S[0][k] + S[1][k] - S[2][k] + S[3][k]); };
    auto Dy = [&](int k) { return hy * (-S[0][k] - S[1][k] + S[2][k] + S[3][k]); };
    const C axx = C(0.5) * Dx(0), axy = Dy(0);
    const C bxy = Dx(1), byy = C(0.5) * Dy(1);
    const C bxx = Dx(2) - C(0.5) * axy, ayy = Dy(2) - C(0.5) * bxy;
    u[0] -= wd * (axx + ayy);
    u[1] -= wd * (bxx + byy);
  }
}

// Reverse of one interpolated ghost.  Inputs: the four source records, the
// linear weights beta, the f^neq rescale r, the target's omega (omega_t) and
// the adjoints of the ghost's post-collision g* (lgs) and, for
// GhostFromFiner, of its own record (lrec, may be null).  Outputs: adjoints
// of the four source records (lsrc[4][stride]) and the omega partials
// (d_t for the target level, d_s for the source level).
template <class Lat, class C>
__device__ __forceinline__ void ghost_adjoint(const C* const* rec, const C* beta, C r, C omega_t,
                                              C omega_s, C rho0, int sx, int sy, int sz, C wd,
                                              C wc, const C* lgs, const C* lrec, C (*lsrc)[cap_stride(Lat::Q)],
                                              double& d_t, double& d_s) {
  constexpr int D = Lat::D, Q = Lat::Q, NS = Lat::NS;
  // forward recompute
  C drho = 0, u[3] = {0, 0, 0}, fneq[Q];
  const C* S[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    drho += beta[k] * rec[k][cap_rho(Lat::Q)];
#pragma unroll
    for (int b = 0; b < D; ++b) u[b] += beta[k] * rec[k][cap_u(Lat::Q) + b];
    S[k] = rec[k] + cap_s(Lat::Q);
  }
  strain_terms<D, C>(S, sx, sy, sz, wd, wc, u);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    C m = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) m += beta[k] * rec[k][cap_fneq(Lat::Q) + i];
    fneq[i] = r * m;
  }
  const C rho = rho0 + drho;
  const C uu = dot_uu<Lat, C>(u);
  // adjoint of g* = g_eq + (1 - omega_t) fneq and of the record
  C lfneq[Q], lgeq[Q];
  C ldrho = 0, lrho = 0, lu[3] = {0, 0, 0};
  double dt = 0, ds = 0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    lgeq[i] = lgs[i];
    lfneq[i] = (C(1) - omega_t) * lgs[i];
    dt -= (double)lgs[i] * (double)fneq[i];
  }
  if (lrec) {
    const C pref = -C(1.5) * omega_t / rho;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      C pi = 0;
#pragma unroll
      for (int i = 0; i < Q; ++i) pi += C(Lat::c(i, strain_a(D, k)) * Lat::c(i, strain_b(D, k))) * fneq[i];
      const C Sk = pref * pi;
      const C lS = lrec[cap_s(Lat::Q) + k];
      lrho -= lS * Sk / rho;
      dt += (double)lS * (double)Sk / (double)omega_t;
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      C lf = lrec[cap_fneq(Lat::Q) + i];
#pragma unroll
      for (int k = 0; k < NS; ++k)
        lf += pref * C(Lat::c(i, strain_a(D, k)) * Lat::c(i, strain_b(D, k))) * lrec[cap_s(Lat::Q) + k];
      lfneq[i] += lf;
    }
    ldrho += lrec[cap_rho(Lat::Q)];
#pragma unroll
    for (int b = 0; b < D; ++b) lu[b] += lrec[cap_u(Lat::Q) + b];
  }
  // rescale r = omega_s dt_t / (omega_t dt_s): d r/d omega_s = r/omega_s,
  // d r/d omega_t = -r/omega_t
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double p = (double)lfneq[i] * (double)fneq[i];
    ds += p / (double)omega_s;
    dt -= p / (double)omega_t;
  }
  geq_adjoint<Lat, C>(lgeq, rho, u, uu, ldrho, lrho, lu);
  ldrho += lrho;
  // to the sources
  C lS[4][6];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int c = 0; c < 6; ++c) lS[k][c] = 0;
  strain_terms_adjoint<D, C>(lu, sx, sy, sz, wd, wc, lS);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    lsrc[k][cap_rho(Lat::Q)] = beta[k] * ldrho;
#pragma unroll
    for (int b = 0; b < D; ++b) lsrc[k][cap_u(Lat::Q) + b] = beta[k] * lu[b];
#pragma unroll
    for (int c = 0; c < NS; ++c) lsrc[k][cap_s(Lat::Q) + c] = lS[k][c];
#pragma unroll
    for (int i = 0; i < Q; ++i) lsrc[k][cap_fneq(Lat::Q) + i] = beta[k] * r * lfneq[i];
  }
  d_t += dt;
  d_s += ds;
}

// GhostFromFiner reverse, one thread per ghost of the coarse level.
template <class Lat, int P>
__global__ __launch_bounds__(64) void k_adj_gff(
    int64_t gff_begin, int64_t n_gff, const int32_t* __restrict__ slots,
    const typename Prec<P>::C* __restrict__ cap_fine, const typename Prec<P>::C* __restrict__ lam,
    int64_t n, typename Prec<P>::C* __restrict__ lam_cap_coarse, int64_t cap_gff_begin,
    typename Prec<P>::C* __restrict__ lam_cap_fine, typename Prec<P>::C omega_c,
    typename Prec<P>::C omega_f, typename Prec<P>::C rho0, double* __restrict__ part) {
  using C = typename Prec<P>::C;
  constexpr int D = Lat::D, Q = Lat::Q;
  __shared__ double sm[DPART];
  const int64_t j = (int64_t)blockIdx.x * 64 + threadIdx.x;
  double acc[DPART] = {0, 0, 0, 0, 0};
  if (j < n_gff) {
    const C* rec[4];
    int32_t sl[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      sl[k] = slots[k * n_gff + j];
      rec[k] = cap_fine + (int64_t)sl[k] * cap_stride(Lat::Q);
    }
    C lgs[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) lgs[i] = lam[(int64_t)i * n + gff_begin + j];
    C* lr = lam_cap_coarse + (cap_gff_begin + j) * cap_stride(Lat::Q);
    C lrec[cap_used(Lat::Q)];
#pragma unroll
    for (int c = 0; c < cap_used(Lat::Q); ++c) {
      lrec[c] = lr[c];
      lr[c] = C(0);
    }
    const C beta[4] = {C(0.25), C(0.25), C(0.25), C(0.25)};
    C lsrc[4][cap_stride(Lat::Q)];
    ghost_adjoint<Lat, C>(rec, beta, C(2) * omega_f / omega_c, omega_c, omega_f, rho0, 1, 1, 1,
                          C(0.25), C(0), lgs, lrec, lsrc, acc[0], acc[1]);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      C* dst = lam_cap_fine + (int64_t)sl[k] * cap_stride(Lat::Q);
#pragma unroll
      for (int c = 0; c < cap_used(Lat::Q); ++c) dst[c] += lsrc[k][c];
    }
  }
  block_sums(sm, acc, DPART, part + (int64_t)blockIdx.x * DPART);
}

// GhostFromCoarser reverse, phase 1.  One work-group takes GPB parent
// groups, one thread per child ghost (as the forward fill); each child forms
// the adjoints of its four source records, and the group sums them per
// neighbourhood slot in LDS, children in a fixed order, before writing one
// row per (group, slot) to T[group][slot][stride].
template <class Lat, int P>
__global__ __launch_bounds__(64) void k_adj_gfc(
    int64_t n_groups, const int32_t* __restrict__ grp_src, const int32_t* __restrict__ grp_child,
    const typename Prec<P>::C* __restrict__ cap_coarse,
    const typename Prec<P>::C* __restrict__ lam, int64_t n, typename Prec<P>::C* __restrict__ T,
    typename Prec<P>::C omega_f, typename Prec<P>::C omega_c, typename Prec<P>::C rho0,
    double* __restrict__ part) {
  using C = typename Prec<P>::C;
  constexpr int D = Lat::D, Q = Lat::Q;
  constexpr int NB = group_slots(D), NC = group_children(D), GPB = 64 / NC;
  constexpr int ST = cap_stride(Q), USED = cap_used(Q);
  __shared__ C sums[GPB * NB * USED];
  __shared__ double sm[DPART];
  for (int e = threadIdx.x; e < GPB * NB * USED; e += 64) sums[e] = C(0);
  const int gl = threadIdx.x / NC, c = threadIdx.x % NC;
  const int64_t g = (int64_t)blockIdx.x * GPB + gl;
  const int32_t target = g < n_groups ? grp_child[(int64_t)c * n_groups + g] : -1;
  double acc[DPART] = {0, 0, 0, 0, 0};
  C lsrc[4][ST];
  int sl[4] = {0, 0, 0, 0};
  if (target >= 0) {
    const int sx = (c & 1) ? 1 : -1, sy = (c & 2) ? 1 : -1, sz = (c & 4) ? 1 : -1;
    C beta[4];
    C wd, wc;
    if constexpr (D == 3) {
      sl[0] = group_slot_of(3, 0, 0, 0);     // H
      sl[1] = group_slot_of(3, sx, sy, 0);   // K
      sl[2] = group_slot_of(3, sx, 0, sz);   // M
      sl[3] = group_slot_of(3, 0, sy, sz);   // N
      beta[0] = C(0.625); beta[1] = beta[2] = beta[3] = C(0.125);
      wd = C(3.0 / 16.0); wc = C(1.0 / 16.0);
    } else {
      sl[0] = group_slot_of(2, 0, 0, 0);     // P
      sl[1] = group_slot_of(2, sx, 0, 0);    // P + s_x
      sl[2] = group_slot_of(2, 0, sy, 0);    // P + s_y
      sl[3] = group_slot_of(2, sx, sy, 0);   // P + s_x + s_y
      beta[0] = C(9.0 / 16.0); beta[1] = beta[2] = C(3.0 / 16.0); beta[3] = C(1.0 / 16.0);
      wd = C(3.0 / 16.0); wc = C(0);
    }
    const C* rec[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      rec[k] = cap_coarse + (int64_t)grp_src[(int64_t)sl[k] * n_groups + g] * ST;
    C lgs[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) lgs[i] = lam[(int64_t)i * n + target];
    ghost_adjoint<Lat, C>(rec, beta, omega_c / (C(2) * omega_f), omega_f, omega_c, rho0, sx, sy,
                          sz, wd, wc, lgs, nullptr, lsrc, acc[0], acc[1]);
  }
  __syncthreads();
  // children of a group add in turn (its four slots are distinct)
  for (int p = 0; p < NC; ++p) {
    if (c == p && target >= 0) {
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int cc = 0; cc < USED; ++cc) sums[(gl * NB + sl[k]) * USED + cc] += lsrc[k][cc];
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < GPB * NB * USED; e += 64) {
    const int g2 = e / (NB * USED), r = e % (NB * USED);
    const int64_t gg = (int64_t)blockIdx.x * GPB + g2;
    if (gg < n_groups) T[(gg * NB + r / USED) * ST + r % USED] = sums[e];
  }
  block_sums(sm, acc, DPART, part + (int64_t)blockIdx.x * DPART);
}

// Phase 2: each coarse record sums its contributions in a fixed order.
template <class Lat, class C>
__global__ __launch_bounds__(256) void k_adj_gfc_gather(const int32_t* __restrict__ ptr,
                                                        const int32_t* __restrict__ ent,
                                                        int64_t n_slots, const C* __restrict__ T,
                                                        C* __restrict__ lam_cap) {
  constexpr int D = Lat::D;
  constexpr int W = cap_used(Lat::Q);
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t s = t / W, c = t % W;
  if (s >= n_slots) return;
  C v = 0;
  for (int32_t e = ptr[s]; e < ptr[s + 1]; ++e) v += T[(int64_t)ent[e] * cap_stride(Lat::Q) + c];
  if (ptr[s + 1] > ptr[s]) lam_cap[s * cap_stride(Lat::Q) + c] += v;
}

// Init reverse: f = f^eq(rho, u) + f^neq(S) per fluid element, collided into
// the stored state and recorded when the element is a source.
template <class Lat, int P>
__global__ __launch_bounds__(256) void k_adj_init(
    const double* __restrict__ rho_in, const double* __restrict__ u_in,
    const double* __restrict__ S_in, int64_t nf, const LevelArgs<typename Prec<P>::C, Lat::Q> a,
    double omega_d, const typename Prec<P>::C* __restrict__ lam,
    typename Prec<P>::C* __restrict__ lam_cap, double* __restrict__ du, double* __restrict__ drho_out,
    double* __restrict__ dS, double* __restrict__ part) {
  using C = typename Prec<P>::C;
  constexpr int D = Lat::D, Q = Lat::Q, NS = Lat::NS;
  __shared__ double sm[4 * DPART];
  const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double acc[DPART] = {0, 0, 0, 0, 0};
  if (x < nf) {
    double gd[Q];
    init_g<Lat>(rho_in, u_in, S_in, nf, x, (double)a.rho0, omega_d, gd);
    C g[Q], ls[Q], mu[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      g[i] = (C)gd[i];
      ls[i] = lam[(int64_t)i * a.n + x];
    }
    const bool src = x >= a.cap_begin;
    C lrec[cap_used(Lat::Q)];
    if (src) {
      C* r = lam_cap + (x - a.cap_begin) * cap_stride(Lat::Q);
#pragma unroll
      for (int c = 0; c < cap_used(Lat::Q); ++c) {
        lrec[c] = r[c];
        r[c] = C(0);
      }
    }
    collide_adjoint<Lat, C>(g, ls, src ? lrec : nullptr, a.rho0, a.omega, mu, acc[0]);
    // f_i = w rho (1 + 3 cu + 4.5 cu^2 - 1.5 uu) - 3 w rho / omega (c c : S - tr S / 3)
    const double rho = rho_in[x];
    double u[3] = {0, 0, 0}, S[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int b = 0; b < D; ++b) u[b] = u_in[(int64_t)b * nf + x];
    if (S_in) {
#pragma unroll
      for (int k = 0; k < NS; ++k) S[k] = S_in[(int64_t)k * nf + x];
    }
    const double uu = dot_uu<Lat, double>(u);
    double trS = 0;
#pragma unroll
    for (int b = 0; b < D; ++b) trS += S[b];
    double lu[3] = {0, 0, 0}, lrho = 0, lS[6] = {0, 0, 0, 0, 0, 0}, dw = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const double m = (double)mu[i], w = Lat::w(i);
      double cu = 0, cSc = 0;
#pragma unroll
      for (int b = 0; b < D; ++b) cu += Lat::c(i, b) * u[b];
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        const int aa = strain_a(D, k), bb = strain_b(D, k);
        cSc += (aa == bb ? 1.0 : 2.0) * Lat::c(i, aa) * Lat::c(i, bb) * S[k];
      }
      const double QS = cSc - trS / 3.0;
      const double feq_over_rho = w * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
      const double fneq = -3.0 * w * rho / omega_d * QS;
      lrho += m * (feq_over_rho + fneq / rho);
      dw += m * (-fneq / omega_d);
#pragma unroll
      for (int b = 0; b < D; ++b)
        lu[b] += m * w * rho * (3.0 * Lat::c(i, b) + 9.0 * cu * Lat::c(i, b) - 3.0 * u[b]);
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        const int aa = strain_a(D, k), bb = strain_b(D, k);
        const double dq = (aa == bb) ? (Lat::c(i, aa) * Lat::c(i, aa) - 1.0 / 3.0)
                                     : 2.0 * Lat::c(i, aa) * Lat::c(i, bb);
        lS[k] += m * (-3.0 * w * rho / omega_d) * dq;
      }
    }
#pragma unroll
    for (int b = 0; b < D; ++b) du[(int64_t)b * nf + x] = lu[b];
    if (drho_out) drho_out[x] = lrho;
    if (dS) {
#pragma unroll
      for (int k = 0; k < NS; ++k) dS[(int64_t)k * nf + x] = lS[k];
    }
    acc[0] += dw;
  }
  block_sums(sm, acc, DPART, part + (int64_t)blockIdx.x * DPART);
}

// [q][ld] in the compute type -> [q][n] FP64 (total = q n entries)
template <class C>
__global__ __launch_bounds__(256) void k_to_double(const C* __restrict__ in, int64_t n,
                                                   int64_t ld, int64_t total,
                                                   double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t < total) out[t] = (double)in[(t / n) * ld + t % n];
}

// Deterministic reduction of all partial records, op by op in a fixed order.
struct AdjOp {
  int64_t offset;   // first block record
  int64_t blocks;
  int32_t level_self, level_other;  // -1 when unused
  int32_t chunk_begin, chunk_count; // its chunks in the first reduction stage
};

// A run of at most REDUCE_CHUNK consecutive block records of one op.
constexpr int REDUCE_CHUNK = 2048;
struct AdjChunk {
  int64_t start;
  int64_t count;
};

// Stage 1: one work-group per chunk sums its records in a fixed order.
__global__ __launch_bounds__(256) void k_adj_reduce_chunks(const double* __restrict__ part,
                                                           const AdjChunk* __restrict__ chunks,
                                                           double* __restrict__ chunk_sums) {
  __shared__ double sm[4 * DPART];
  const AdjChunk c = chunks[blockIdx.x];
  double v[DPART] = {0, 0, 0, 0, 0};
  for (int64_t b = threadIdx.x; b < c.count; b += 256)
#pragma unroll
    for (int k = 0; k < DPART; ++k) v[k] += part[(c.start + b) * DPART + k];
  block_sums(sm, v, DPART, chunk_sums + (int64_t)blockIdx.x * DPART);
}

// Stage 2: one thread adds each op's chunk sums, op by op, into the
// parameter accumulators.
__global__ __launch_bounds__(64) void k_adj_reduce(const double* __restrict__ chunk_sums,
                                                   const AdjOp* __restrict__ ops, int n_ops,
                                                   double* __restrict__ acc, int nlev) {
  if (threadIdx.x != 0) return;
  for (int o = 0; o < n_ops; ++o) {
    const AdjOp op = ops[o];
    double tot[DPART] = {0, 0, 0, 0, 0};
    for (int c = 0; c < op.chunk_count; ++c)
#pragma unroll
      for (int k = 0; k < DPART; ++k) tot[k] += chunk_sums[(int64_t)(op.chunk_begin + c) * DPART + k];
    if (op.level_self >= 0) acc[op.level_self] += tot[0];
    if (op.level_other >= 0) acc[op.level_other] += tot[1];
    for (int k = 0; k < 3; ++k) acc[nlev + k] += tot[2 + k];
  }
}

}  // namespace mlbm
