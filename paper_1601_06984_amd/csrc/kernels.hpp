// Forward device kernels: fused pull stream-collide, source capture, the
// GhostFromFiner / GhostFromCoarser compact-interpolation fills, init,
// state conversion and FP64 diagnostics.
//
// All arithmetic works on deviations g_i = f_i - w_i rho0 (exact for the
// F64 stored values by Sterbenz' lemma; the stored form of F32 and F16S),
// which keeps FP32 rounding relative to the small deviations instead of
// to the O(1) pdfs.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include "common.hpp"

namespace mlbm {

// ---------------------------------------------------------------- storage --
// Stored value of g_i = f_i - w_i rho0: F64 keeps f itself (its rounding is
// far below anything the method resolves); F32 keeps the deviation g, whose
// rounding is relative to O(u) values instead of to f ~ w_i; F16S keeps
// fp16(s_L g).
template <int P> struct Prec;
template <> struct Prec<MLBM_F64> { using S = double; using C = double; };
template <> struct Prec<MLBM_F32> { using S = float; using C = float; };
template <> struct Prec<MLBM_F16S> { using S = __half; using C = float; };

template <int P>
__device__ __forceinline__ typename Prec<P>::C load_g(const typename Prec<P>::S* __restrict__ p,
                                                     int64_t idx, typename Prec<P>::C wr,
                                                     typename Prec<P>::C inv_scale) {
  if constexpr (P == MLBM_F16S) {
    (void)wr;
    return __half2float(p[idx]) * inv_scale;
  } else if constexpr (P == MLBM_F32) {
    (void)wr;
    (void)inv_scale;
    return p[idx];
  } else {
    (void)inv_scale;
    return (typename Prec<P>::C)p[idx] - wr;
  }
}

template <int P>
__device__ __forceinline__ bool store_g(typename Prec<P>::S* __restrict__ p, int64_t idx,
                                        typename Prec<P>::C g, typename Prec<P>::C wr,
                                        typename Prec<P>::C scale) {
  if constexpr (P == MLBM_F16S) {
    (void)wr;
    const float h = g * scale;
    p[idx] = __float2half_rn(h);
    return fabsf(h) <= 65504.0f;
  } else if constexpr (P == MLBM_F32) {
    (void)wr;
    (void)scale;
    p[idx] = g;
    return true;
  } else {
    (void)scale;
    p[idx] = (typename Prec<P>::S)(wr + g);
    return true;
  }
}

// Row access through buffer instructions: a wave-uniform row start and
// length give a scalar buffer descriptor, each lane supplies a 32-bit byte
// offset (no 64-bit address arithmetic per lane), and the hardware drops
// stores and zeroes loads outside the row.  Rows stay below 4 GiB (checked
// at sim_create).  0x00020000 is the gfx9-family descriptor word 3 for
// untyped 32-bit data.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const void* row, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(row), (short)0, (int)(uint32_t)bytes,
                                           0x00020000);
}

__device__ __forceinline__ int32_t load_idx(const int32_t* row, int64_t len, uint32_t e) {
  return __builtin_amdgcn_raw_buffer_load_b32(row_rsrc(row, len * 4), (int)(e * 4u), 0, 0);
}

template <class S>
__device__ __forceinline__ S load_elem(const S* row, int64_t len, uint32_t e) {
  const auto r = row_rsrc(row, len * (int64_t)sizeof(S));
  const int off = (int)(e * (uint32_t)sizeof(S));
  if constexpr (sizeof(S) == 8)
    return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
  else if constexpr (sizeof(S) == 4)
    return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
  else
    return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0));
}

template <class S>
__device__ __forceinline__ void store_elem(S* row, int64_t len, uint32_t e, S v) {
  const auto r = row_rsrc(row, len * (int64_t)sizeof(S));
  const int off = (int)(e * (uint32_t)sizeof(S));
  if constexpr (sizeof(S) == 8) {
    typedef int v2i __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2i, v), r, off, 0, 0);
  } else if constexpr (sizeof(S) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, v), r, off, 0, 0);
  } else {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(short, v), r, off, 0, 0);
  }
}

template <int P>
__device__ __forceinline__ typename Prec<P>::C load_row(const typename Prec<P>::S* __restrict__ row,
                                                        int64_t len, uint32_t e,
                                                        typename Prec<P>::C wr,
                                                        typename Prec<P>::C inv_scale) {
  if constexpr (P == MLBM_F16S) {
    (void)wr;
    return __half2float(load_elem(row, len, e)) * inv_scale;
  } else if constexpr (P == MLBM_F32) {
    (void)wr;
    (void)inv_scale;
    return load_elem(row, len, e);
  } else {
    (void)inv_scale;
    return (typename Prec<P>::C)load_elem(row, len, e) - wr;
  }
}

template <int P>
__device__ __forceinline__ bool store_row(typename Prec<P>::S* __restrict__ row, int64_t len,
                                          uint32_t e, typename Prec<P>::C g,
                                          typename Prec<P>::C wr, typename Prec<P>::C scale) {
  using S = typename Prec<P>::S;
  if constexpr (P == MLBM_F16S) {
    (void)wr;
    const float h = g * scale;
    store_elem(row, len, e, __float2half_rn(h));
    return fabsf(h) <= 65504.0f;
  } else if constexpr (P == MLBM_F32) {
    (void)wr;
    (void)scale;
    store_elem(row, len, e, (S)g);
    return true;
  } else {
    (void)scale;
    store_elem(row, len, e, (S)(wr + g));
    return true;
  }
}

// Per-level parameters passed by value.
template <class C, int Q>
struct LevelArgs {
  int64_t n;          // row stride of the [q][n] pdf arrays (the level's padded stride)
  // pull table, device form (see the plan's NBR16 table): 16-bit codes
  // [q-1][ld16], bases [blocks][q-1][NBR_BASES], wide rows [q-1][ldw]
  const uint16_t* nbr16;
  const int32_t* nbase;
  const uint16_t* nbr_wide;
  const int32_t* nhdr;  // [blocks][NBR_HDR]
  int32_t morton;       // nonzero: blocks may hold Morton directions
  int64_t ld16, ldw;
  int64_t cap_begin;  // fluid elements [cap_begin, n_fluid) are sources
  int64_t n_fluid;
  C omega;            // BGK relaxation rate of the level
  C rho0;
  C scale, inv_scale; // F16S scale s_L and 1/s_L
  C wr[4];            // w_i rho0 per weight class (Lat::wclass)
  const C* geq;       // device [Q]: f^eq_i(rho0, u_in) - w_i rho0 for EQ faces
  double u_in[3];     // EQ-face velocity
  // links with a wall fraction, sorted by element: {x, j, x2, weight class},
  // and their fractions (null: none on the level)
  const int4* wall;
  const double* wall_q;
  int32_t n_wall;
};

// -------------------------------------------------------- BGK in g-form ---
// rho = rho0 + sum g; rho u = sum c g; g_eq = w (drho + rho (3 cu + 4.5 cu^2 - 1.5 uu))
template <class Lat, class C>
__device__ __forceinline__ void macro_g(const C* g, C rho0, C& drho, C& rho, C* u) {
  C s = 0, j[3] = {0, 0, 0};
#pragma unroll
  for (int i = 0; i < Lat::Q; ++i) {
    s += g[i];
#pragma unroll
    for (int a = 0; a < Lat::D; ++a) {
      const int ci = Lat::c(i, a);
      if (ci > 0) j[a] += g[i];
      if (ci < 0) j[a] -= g[i];
    }
  }
  drho = s;
  rho = rho0 + s;
  const C inv = C(1) / rho;
#pragma unroll
  for (int a = 0; a < 3; ++a) u[a] = a < Lat::D ? j[a] * inv : C(0);
}

// macro_g of FP32 deviations accumulated in FP64
template <class Lat>
__device__ __forceinline__ void macro_g_wide(const float* g, double rho0, double& drho,
                                             double& rho, double* u) {
  double s = 0, j[3] = {0, 0, 0};
#pragma unroll
  for (int i = 0; i < Lat::Q; ++i) {
    const double gi = g[i];
    s += gi;
#pragma unroll
    for (int a = 0; a < Lat::D; ++a) {
      const int ci = Lat::c(i, a);
      if (ci > 0) j[a] += gi;
      if (ci < 0) j[a] -= gi;
    }
  }
  drho = s;
  rho = rho0 + s;
  const double inv = 1.0 / rho;
#pragma unroll
  for (int a = 0; a < 3; ++a) u[a] = a < Lat::D ? j[a] * inv : 0.0;
}

template <class Lat, class C>
__device__ __forceinline__ C geq_i(int i, C drho, C rho, const C* u, C uu) {
  C cu = 0;
#pragma unroll
  for (int a = 0; a < Lat::D; ++a) {
    const int ci = Lat::c(i, a);
    if (ci > 0) cu += u[a];
    if (ci < 0) cu -= u[a];
  }
  const C w = (C)Lat::w(i);
  return w * (drho + rho * (C(3) * cu + C(4.5) * cu * cu - C(1.5) * uu));
}

template <class Lat, class C>
__device__ __forceinline__ C dot_uu(const C* u) {
  C s = 0;
#pragma unroll
  for (int a = 0; a < Lat::D; ++a) s += u[a] * u[a];
  return s;
}

// ------------------------------------------------------ pull gather ------
// g_i(x) = g*_i(nbr_i(x)) with boundary codes: BOUNCE -> g*_opp(i)(x),
// COPY -> g*_i(x), EQ -> f^eq(rho0, u_in).  MISSING never occurs in an
// updated range: the planner rejects meshes where it would.
__device__ __forceinline__ uint32_t load_u16(const uint16_t* row, int64_t len, uint32_t e) {
  return (uint32_t)(uint16_t)__builtin_amdgcn_raw_buffer_load_b16(row_rsrc(row, len * 2),
                                                                  (int)(e * 2u), 0, 0);
}

// Source index (or link code) of a 16-bit pull code against the four bases
// of its block and direction.
__device__ __forceinline__ int32_t pull_decode(uint32_t c, int32_t b0, int32_t b1, int32_t b2,
                                               int32_t b3) {
  const uint32_t s = c >> 14;
  const int32_t base = s == 0 ? b0 : (s == 1 ? b1 : (s == 2 ? b2 : b3));
  return c >= NBR_CODE0 ? (int32_t)c - 0x10000 : base + (int32_t)(c & 0x3FFFu);
}

// Source of a Morton direction (see LevelPlan): the Morton code of x - c_i
// shifted by the constant of its run; {k0, k1, t0, t1} are the slot values.
template <class Lat>
__device__ __forceinline__ int32_t morton_source(uint32_t m, int i, int32_t k0, int32_t k1,
                                                 int32_t t0, int32_t t1) {
  const uint32_t mo = morton_pull<Lat>(m, i);
  return (int32_t)(mo + ((mo - (uint32_t)t0) >= (uint32_t)t1 ? (uint32_t)k1 : (uint32_t)k0));
}

// Pull sources j[1..Q-1] of element x in pull-table block blk (x >> 8).
// Kernels whose work-groups cover whole blocks pass a block index that is
// uniform over the work-group, so the header and slots come through scalar
// loads.  Directions whose sources follow from Morton arithmetic read no
// codes (their lanes load past the end of the row, which the buffer range
// check answers with 0 and no memory access).  Both readings of a slot are
// formed and one is kept by a mask, without branches, so that the code
// loads of all directions are in flight together.
template <class Lat, int MODE, class LA>
__device__ __forceinline__ void pull_sources_mode(const LA& a, int64_t blk, uint32_t x,
                                                  uint32_t regm, uint32_t m, int32_t* j) {
  // MODE 0: every direction decodes its code; 1: every direction is a
  // Morton direction; 2: the mask regm chooses per direction
  constexpr int Q = Lat::Q;
  const int32_t* __restrict__ bb = a.nbase + blk * (Q - 1) * NBR_BASES;
  int32_t s[Q][NBR_BASES];
#pragma unroll
  for (int i = 1; i < Q; ++i)
#pragma unroll
    for (int t = 0; t < NBR_BASES; ++t) s[i][t] = bb[(i - 1) * NBR_BASES + t];
  uint32_t c[Q];
  if constexpr (MODE != 1) {
#pragma unroll
    for (int i = 1; i < Q; ++i)
      c[i] = load_u16(a.nbr16 + (int64_t)(i - 1) * a.ld16, a.ld16,
                      (MODE == 2 && ((regm >> i) & 1u)) ? NBR_NO_CODE : x);
  }
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    if constexpr (MODE == 0) {
      j[i] = pull_decode(c[i], s[i][0], s[i][1], s[i][2], s[i][3]);
    } else if constexpr (MODE == 1) {
      j[i] = morton_source<Lat>(m, i, s[i][0], s[i][1], s[i][2], s[i][3]);
    } else {
      const uint32_t keep = 0u - ((regm >> i) & 1u);
      const uint32_t jm = (uint32_t)morton_source<Lat>(m, i, s[i][0], s[i][1], s[i][2], s[i][3]);
      const uint32_t jc = (uint32_t)pull_decode(c[i], s[i][0], s[i][1], s[i][2], s[i][3]);
      j[i] = (int32_t)((jm & keep) | (jc & ~keep));
    }
  }
  if constexpr (MODE == 0) {
    const int32_t w = a.nhdr[blk * NBR_HDR + 2];
    if (w >= 0) {   // wide block: codes are the low halves of int32 entries
      const uint32_t e = (uint32_t)w * NBR_BLOCK + (x & (NBR_BLOCK - 1));
#pragma unroll
      for (int i = 1; i < Q; ++i)
        j[i] = (int32_t)((load_u16(a.nbr_wide + (int64_t)(i - 1) * a.ldw, a.ldw, e) << 16) | c[i]);
    }
  }
}

// Pull sources j[1..Q-1] of element x in pull-table block blk (x >> 8).
// Kernels whose work-groups cover whole blocks pass a block index that is
// uniform over the work-group, so the header and slots come through scalar
// loads and the choice below is a branch of the whole wave.  Directions
// whose sources follow from Morton arithmetic read no codes (in a mixed
// block their lanes load past the end of the row, which the buffer range
// check answers with 0 and no memory access); a mixed block forms both
// readings of a slot and keeps one by a mask, without branches, so that the
// code loads of all directions are in flight together.
template <class Lat, class LA>
__device__ __forceinline__ void pull_sources(const LA& a, int64_t blk, uint32_t x, int32_t* j) {
  constexpr uint32_t ALL = (1u << Lat::Q) - 2u;
  if (!a.morton) {   // the level's blocks all decode codes: no header wait
    pull_sources_mode<Lat, 0>(a, blk, x, 0u, 0u, j);
    return;
  }
  const int32_t* __restrict__ hd = a.nhdr + blk * NBR_HDR;
  const uint32_t regm = (uint32_t)hd[0];
  const uint32_t m = x + (uint32_t)hd[1];
  if (regm == 0)
    pull_sources_mode<Lat, 0>(a, blk, x, regm, m, j);
  else if (regm == ALL)
    pull_sources_mode<Lat, 1>(a, blk, x, regm, m, j);
  else
    pull_sources_mode<Lat, 2>(a, blk, x, regm, m, j);
}

// Work-group form of pull_sources: every thread of the work-group calls it
// with the same block.  The block's slots (NBR_SLOTS ints) are staged in
// LDS by the first threads while the code loads are in flight, and each
// lane reads the one base it needs from LDS: no scalar registers hold the
// 4 (q-1) slot values.
constexpr int NBR_SLOTS = 26 * NBR_BASES;   // D3Q27; smaller lattices use a prefix
template <class Lat, int MODE, class LA>
__device__ __forceinline__ void pull_sources_wg_mode(const LA& a, int64_t blk, uint32_t x,
                                                     uint32_t regm, uint32_t m, int32_t* j,
                                                     int32_t* __restrict__ sl) {
  constexpr int Q = Lat::Q, NSL = (Q - 1) * NBR_BASES;
  static_assert(NSL <= NBR_SLOTS && NSL <= 256, "slots fit the staging area");
  uint32_t c[Q];
  if constexpr (MODE == 0) {
#pragma unroll
    for (int i = 1; i < Q; ++i)
      c[i] = load_u16(a.nbr16 + (int64_t)(i - 1) * a.ld16, a.ld16, x);
  } else if constexpr (MODE == 2) {
    // regm is uniform over the work-group: each code load sits behind a
    // scalar branch, so the Morton directions issue no memory instruction;
    // nothing inside the branches uses a loaded value, so the loads of all
    // code directions are still in flight together
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      c[i] = 0u;
      if (!((regm >> i) & 1u)) c[i] = load_u16(a.nbr16 + (int64_t)(i - 1) * a.ld16, a.ld16, x);
    }
  }
  if (threadIdx.x < NSL) sl[threadIdx.x] = a.nbase[blk * NSL + threadIdx.x];
  __syncthreads();
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const int o = (i - 1) * NBR_BASES;
    if constexpr (MODE == 0) {
      j[i] = c[i] >= NBR_CODE0 ? (int32_t)c[i] - 0x10000
                               : sl[o + (int)(c[i] >> 14)] + (int32_t)(c[i] & 0x3FFFu);
    } else {
      const uint32_t mo = morton_pull<Lat>(m, i);
      const uint32_t sm = (mo - (uint32_t)sl[o + 2]) >= (uint32_t)sl[o + 3] ? 1u : 0u;
      if constexpr (MODE == 1) {
        j[i] = (int32_t)(mo + (uint32_t)sl[o + (int)sm]);
      } else {
        const uint32_t keep = 0u - ((regm >> i) & 1u);
        const uint32_t idx = (sm & keep) | ((c[i] >> 14) & ~keep);
        const uint32_t off = (mo & keep) | ((c[i] & 0x3FFFu) & ~keep);
        const int32_t v = (int32_t)((uint32_t)sl[o + (int)idx] + off);
        j[i] = c[i] >= NBR_CODE0 ? (int32_t)c[i] - 0x10000 : v;   // Morton lanes read c = 0
      }
    }
  }
  if constexpr (MODE == 0) {
    const int32_t w = a.nhdr[blk * NBR_HDR + 2];
    if (w >= 0) {   // wide block: codes are the low halves of int32 entries
      const uint32_t e = (uint32_t)w * NBR_BLOCK + (x & (NBR_BLOCK - 1));
#pragma unroll
      for (int i = 1; i < Q; ++i)
        j[i] = (int32_t)((load_u16(a.nbr_wide + (int64_t)(i - 1) * a.ldw, a.ldw, e) << 16) | c[i]);
    }
  }
}

template <class Lat, class LA>
__device__ __forceinline__ void pull_sources_wg(const LA& a, int64_t blk, uint32_t x, int32_t* j,
                                                int32_t* __restrict__ sl) {
  constexpr uint32_t ALL = (1u << Lat::Q) - 2u;
  if (!a.morton) {
    pull_sources_wg_mode<Lat, 0>(a, blk, x, 0u, 0u, j, sl);
    return;
  }
  const int32_t* __restrict__ hd = a.nhdr + blk * NBR_HDR;
  const uint32_t regm = (uint32_t)hd[0];
  const uint32_t m = x + (uint32_t)hd[1];
  if (regm == 0)
    pull_sources_wg_mode<Lat, 0>(a, blk, x, regm, m, j, sl);
  else if (regm == ALL)
    pull_sources_wg_mode<Lat, 1>(a, blk, x, regm, m, j, sl);
  else
    pull_sources_wg_mode<Lat, 2>(a, blk, x, regm, m, j, sl);
}

// Pull source of direction i only.
template <class Lat, class LA>
__device__ __forceinline__ int32_t pull_source(const LA& a, int64_t blk, uint32_t x, int i) {
  const int32_t* __restrict__ hd = a.nhdr + blk * NBR_HDR;
  const int32_t* b = a.nbase + (blk * (Lat::Q - 1) + (i - 1)) * NBR_BASES;
  if (a.morton && (((uint32_t)hd[0] >> i) & 1u))
    return morton_source<Lat>(x + (uint32_t)hd[1], i, b[0], b[1], b[2], b[3]);
  const uint32_t c = load_u16(a.nbr16 + (int64_t)(i - 1) * a.ld16, a.ld16, x);
  int32_t v = pull_decode(c, b[0], b[1], b[2], b[3]);
  const int32_t w = hd[2];
  if (w >= 0)
    v = (int32_t)((load_u16(a.nbr_wide + (int64_t)(i - 1) * a.ldw, a.ldw,
                            (uint32_t)w * NBR_BLOCK + (x & (NBR_BLOCK - 1))) << 16) | c);
  return v;
}

// The pulled values g_i(x) for the sources j[1..Q-1] of element x.
template <class Lat, int P>
__device__ __forceinline__ void gather_from(const typename Prec<P>::S* __restrict__ src, int64_t x,
                                            const LevelArgs<typename Prec<P>::C, Lat::Q>& a,
                                            const int32_t* j, typename Prec<P>::C* g) {
  using C = typename Prec<P>::C;
  const uint32_t xo = (uint32_t)x;
  static_assert(opposite_weights_equal<Lat>(), "w(opp(i)) == w(i)");
  g[0] = load_row<P>(src, a.n, xo, a.wr[0], a.inv_scale);
  const uint32_t nn = (uint32_t)a.n;
  uint32_t eqm = 0;   // directions pulled from an EQ face
#pragma unroll
  for (int i = 1; i < Lat::Q; ++i) {
    // rows 2k-1 and 2k hold opposite directions: one descriptor over the
    // pair serves both the pull (row i) and halfway bounce-back (row
    // opp(i) at x) without a per-lane choice of base address; opposite
    // directions have equal weights, so one weight fits both
    const int pair = (i & 1) ? i : i - 1;
    const int32_t v = j[i];
    const uint32_t e = v >= 0 ? (uint32_t)v : xo;
    const uint32_t off = v == MLBM_NBR_BOUNCE ? (uint32_t)(Lat::opp(i) - pair) * nn + xo
                                             : (uint32_t)(i - pair) * nn + e;
    g[i] = load_row<P>(src + (int64_t)pair * a.n, 2 * a.n, off, a.wr[Lat::wclass(i)], a.inv_scale);
    eqm |= (v == MLBM_NBR_EQ ? 1u : 0u) << i;
  }
  // elements next to an EQ face (few): the face's equilibrium replaces what
  // the lanes loaded (their own entry); the values are read only here, so
  // they hold no registers in the common path
  if (eqm) {
#pragma unroll
    for (int i = 1; i < Lat::Q; ++i)
      if ((eqm >> i) & 1u) g[i] = a.geq[i];
  }
}

// Links that carry a wall fraction q (linear interpolated bounce-back,
// Sec. 2.3): the value pulled in direction j, whose source x - c_j is solid,
// is, with o = opp(j) the direction into the wall,
//   q <  1/2: 2q g*_o(x) + (1 - 2q) g*_o(x2)   (x2 = x + c_j; none: g*_o(x))
//   q >= 1/2: g*_o(x) / (2q) + (1 - 1/(2q)) g*_j(x)
// The weights of each rule sum to one and w_o = w_j, so the rule holds for
// the deviations g = f - w rho0 as for f.
//
// Before a stream-collide of a level with such links this kernel writes
// each link's value into the entry that the halfway bounce-back pull of the
// link reads, g*_o(x): no other pull reads that entry (its pull would come
// from x + c_o = x - c_j, which is solid), and the stream-collide then
// gathers the interpolated value with no code of its own for the links.
// The entry belongs to the state the stream-collide consumes and replaces.
// One thread per link; every value is formed before any is written.  The
// entries read are x's own and g*_o(x2); none written for another element
// (x2 is fluid, and g*_o(x2) would be written only by a link of x2 in
// direction j, whose solid source would be x).  Within an element, g*_j(x)
// is read where the opposite link writes (an element between two walls);
// an element's links lie in one chunk of 256 (the list is padded with
// links x = -1), so the work-group barrier orders them.
template <class Lat, class C>
__device__ __forceinline__ C wall_weight(const LevelArgs<C, Lat::Q>& a, int cls) {
  C w = a.wr[0];
  if (cls == 1) w = a.wr[1];
  if (cls == 2) w = a.wr[2];
  if (cls == 3) w = a.wr[3];
  return w;
}

template <class Lat, int P>
__global__ __launch_bounds__(256) void k_wall_prepass(
    typename Prec<P>::S* __restrict__ src, const LevelArgs<typename Prec<P>::C, Lat::Q> a) {
  using C = typename Prec<P>::C;
  const int32_t t = (int32_t)(blockIdx.x * 256 + threadIdx.x);
  int4 w = {-1, 0, -1, 0};
  if (t < a.n_wall) w = a.wall[t];
  const int jd = w.y;
  const int o = (jd & 1) ? jd + 1 : jd - 1;   // rows 2k-1, 2k are opposite
  const C wr = wall_weight<Lat, C>(a, w.w);
  C v = C(0);
  if (w.x >= 0) {
    const C go = load_row<P>(src + (int64_t)o * a.n, a.n, (uint32_t)w.x, wr, a.inv_scale);
    const C q = (C)a.wall_q[t];
    v = go;
    if (q < C(0.5)) {
      if (w.z >= 0)
        v = C(2) * q * go +
            (C(1) - C(2) * q) * load_row<P>(src + (int64_t)o * a.n, a.n, (uint32_t)w.z, wr,
                                            a.inv_scale);
    } else {
      const C gj = load_row<P>(src + (int64_t)jd * a.n, a.n, (uint32_t)w.x, wr, a.inv_scale);
      const C r = C(1) / (C(2) * q);
      v = r * go + (C(1) - r) * gj;
    }
  }
  __syncthreads();
  // a convex combination of stored values: F16S cannot overflow
  if (w.x >= 0) (void)store_row<P>(src + (int64_t)o * a.n, a.n, (uint32_t)w.x, v, wr, a.scale);
}

template <class Lat, int P>
__device__ __forceinline__ void gather_g(const typename Prec<P>::S* __restrict__ src, int64_t blk,
                                         int64_t x,
                                         const LevelArgs<typename Prec<P>::C, Lat::Q>& a,
                                         typename Prec<P>::C* g) {
  int32_t j[Lat::Q];
  pull_sources<Lat>(a, blk, (uint32_t)x, j);
  gather_from<Lat, P>(src, x, a, j, g);
}

// Writes the values of one record in slot order with 16-byte stores: each
// put(c, v) must come in increasing c starting from 0; a chunk is stored as
// soon as it is full, and finish() zero-pads and stores the last one.  The
// record base is 16-byte aligned (records start at multiples of 64 bytes).
template <class R>
struct RecordWriter {
  static constexpr int V = 16 / (int)sizeof(R);
  typedef R VT __attribute__((ext_vector_type(16 / sizeof(R))));
  R* __restrict__ p;
  VT buf;
  __device__ __forceinline__ void put(int c, R v) {
    buf[c % V] = v;
    if (c % V == V - 1) *reinterpret_cast<VT*>(p + (c - (V - 1))) = buf;
  }
  __device__ __forceinline__ void finish(int used) {
    if (used % V) {
#pragma unroll
      for (int c = used % V; c < V; ++c) buf[c] = R(0);
      *reinterpret_cast<VT*>(p + (used - used % V)) = buf;
    }
  }
};

// The values of a capture record in slot order: g^neq, drho, u,
// S_ab = -(3 omega / (2 rho)) sum_i c_ia c_ib g^neq_i, handed to a writer
// (RecordWriter or WaveRecordStager) one slot at a time.
template <class Lat, class C, class Wr>
__device__ __forceinline__ void record_values(Wr& w, const C* g, C drho, C rho, const C* u, C uu,
                                              C omega) {
  constexpr int D = Lat::D;
  static_assert(cap_fneq(Lat::Q) == 0 && cap_rho(Lat::Q) == Lat::Q, "record layout");
  // streamed: each g^neq_i is handed on and folded into the second moments
  // as it is formed, so no per-direction array stays live
  C pi[Lat::NS];
#pragma unroll
  for (int k = 0; k < Lat::NS; ++k) pi[k] = C(0);
#pragma unroll
  for (int i = 0; i < Lat::Q; ++i) {
    const C fneq = g[i] - geq_i<Lat, C>(i, drho, rho, u, uu);
    w.put(cap_fneq(Lat::Q) + i, fneq);
#pragma unroll
    for (int k = 0; k < Lat::NS; ++k) {
      const int cc = Lat::c(i, strain_a(D, k)) * Lat::c(i, strain_b(D, k));
      if (cc > 0) pi[k] += fneq;
      if (cc < 0) pi[k] -= fneq;
    }
  }
  w.put(cap_rho(Lat::Q), drho);
#pragma unroll
  for (int a = 0; a < D; ++a) w.put(cap_u(Lat::Q) + a, u[a]);
  const C pref = -C(1.5) * omega / rho;
#pragma unroll
  for (int k = 0; k < Lat::NS; ++k) w.put(cap_s(Lat::Q) + k, pref * pi[k]);
  w.finish(cap_used(Lat::Q));
}

template <class Lat, class C, class R>
__device__ __forceinline__ void write_record_m(R* __restrict__ rec, const C* g, C drho, C rho,
                                               const C* u, C uu, C omega) {
  RecordWriter<R> w{rec, {}};   // values rounded to the record type
  record_values<Lat, C>(w, g, drho, rho, u, uu, omega);
}

// Capture records of a whole wavefront, staged through LDS.  Each record is
// written in phases of 64 bytes: the lanes put their values of the phase
// into their LDS rows, then the wave stores the phase of all its source
// records with 16-byte stores, four consecutive lanes covering one record's
// 64 contiguous bytes (instead of every lane's stores touching 64 lines).
// All 64 lanes call put/finish together (wave-uniform control flow); bit r
// of `mask` marks lane r as a source, whose record is rbase + r.  LDS ops of
// one wave complete in order; the wavefront fences keep the compiler from
// moving them across the phase boundary.
template <class C, int ST>
struct WaveRecordStager {
  static constexpr int V = 16 / (int)sizeof(C);   // values per 16-byte chunk
  static constexpr int PH = 64 / (int)sizeof(C);  // values per phase
  static constexpr int RS = PH + V;               // LDS row stride, 16-byte aligned
  static constexpr int LDS_PER_WAVE = 64 * RS;    // values
  static_assert(ST % PH == 0, "record stride");
  typedef C VT __attribute__((ext_vector_type(16 / sizeof(C))));
  C* __restrict__ lds;   // this wave's 64 rows
  C* __restrict__ cap;   // record array
  int64_t rbase;         // record index of lane 0 (only used for set bits)
  uint64_t mask;
  int lane;
  VT buf;
  __device__ __forceinline__ void put(int c, C v) {
    buf[c % V] = v;
    if (c % V == V - 1) {
      *reinterpret_cast<VT*>(lds + lane * RS + (c % PH) - (V - 1)) = buf;
      if (c % PH == PH - 1) flush(c - (PH - 1));
    }
  }
  __device__ __forceinline__ void flush(int c0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int t = 0; t < 4; ++t) {          // 64 records x 4 chunks of 16 bytes
      const int q = t * 64 + lane, r = q >> 2, ch = q & 3;
      if ((mask >> r) & 1ull) {
        const VT v = *reinterpret_cast<const VT*>(lds + r * RS + ch * V);
        *reinterpret_cast<VT*>(cap + (rbase + r) * ST + c0 + ch * V) = v;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  __device__ __forceinline__ void finish(int used) {
#pragma unroll
    for (int c = used; c < (used + PH - 1) / PH * PH; ++c) put(c, C(0));
  }
};

template <class Lat, class C, class R>
__device__ __forceinline__ void write_record(R* __restrict__ rec, const C* g, C rho0, C omega) {
  C drho, rho, u[3];
  macro_g<Lat, C>(g, rho0, drho, rho, u);
  write_record_m<Lat, C, R>(rec, g, drho, rho, u, dot_uu<Lat, C>(u), omega);
}

// --------------------------------------------------- stream-collide -------
// One thread per element x in [x0, x1); Eq. bgk in g-form, result stored
// coalesced in the destination array.  In the REC instantiation the fluid
// elements of the capture segment also write their pre-collision moments
// (the interpolation input).  Blocks are remapped (xcd_block, xcd_block2)
// so that each of the 8 XCDs streams contiguous slices of the element range.

// Launch on `st`.  With events, they take the kernel's own dispatch start
// and end timestamps (no extra packets between kernels).
template <typename... KArgs, typename... Args>
inline void launch_timed(void (*kernel)(KArgs...), dim3 grid, dim3 block, hipStream_t st,
                         hipEvent_t e0, hipEvent_t e1, Args... args) {
  if (e0 || e1)
    hipExtLaunchKernelGGL(kernel, grid, block, 0, st, e0, e1, 0u, static_cast<KArgs>(args)...);
  else
    hipLaunchKernelGGL(kernel, grid, block, 0, st, static_cast<KArgs>(args)...);
}

// FP16-shift stores of one element's post-collision values that keep the
// element's stored mass and momentum as close to the exact ones as the
// format allows: the diagonal directions round to nearest; each axis pair
// (+a, -a) takes the momentum rounding error along a accumulated so far,
// half on each (antisymmetric, so their mass is unchanged); the rest
// direction takes the accumulated mass error.  What remains is the
// rounding of those last values, instead of the sum over all directions.
// Directions are ordered rest, axis pairs 2a+1 / 2a+2, then diagonals.
// `sink(i, h)` receives the half of direction i (a store to the pdf array,
// or to the work-group's store tile).
template <class Lat, class Sink>
__device__ __forceinline__ bool store_f16s_conserving(Sink&& sink,
                                                      const LevelArgs<float, Lat::Q>& a,
                                                      const float* g, float drho, float rho,
                                                      const float* u, float uu) {
  constexpr int D = Lat::D, Q = Lat::Q;
  bool ok = true;
  // stores round(v) in direction i; returns the decoded value
  auto put = [&](int i, float v) -> float {
    const float hs = v * a.scale;
    const __half h = __float2half_rn(hs);
    sink(i, h);
    ok &= fabsf(hs) <= 65504.0f;
    return __half2float(h) * a.inv_scale;
  };
  auto post = [&](int i) -> float {
    return g[i] + a.omega * (geq_i<Lat, float>(i, drho, rho, u, uu) - g[i]);
  };
  float em = 0.0f, ej[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int i = 2 * D + 1; i < Q; ++i) {
    const float v = post(i);
    const float err = put(i, v) - v;
    em += err;
#pragma unroll
    for (int b = 0; b < D; ++b) ej[b] += (float)Lat::c(i, b) * err;
  }
#pragma unroll
  for (int b = 0; b < D; ++b) {
    const float vp = post(2 * b + 1), vm = post(2 * b + 2);
    const float ep = put(2 * b + 1, vp - 0.5f * ej[b]) - vp;
    const float eq = put(2 * b + 2, vm + 0.5f * ej[b]) - vm;
    em += ep + eq;
  }
  const float v0 = post(0);
  put(0, v0 - em);
  return ok;
}

// The stream-collide of work-group `blk` (blk*BS < x1) of a level whose
// updated range is [0, x1): elements blk*BS .. blk*BS+BS-1.  `stage` is the
// work-group's record staging area, `slots` its pull-table slot area; every
// thread of the work-group calls it.
template <class Lat, int P, int BS>
__device__ __forceinline__ void sc_body(int64_t blk, int64_t x1,
                                        const typename Prec<P>::S* __restrict__ src,
                                        typename Prec<P>::S* __restrict__ dst,
                                        const LevelArgs<typename Prec<P>::C, Lat::Q>& a,
                                        typename Prec<P>::C* __restrict__ cap,
                                        uint32_t* __restrict__ status,
                                        typename Prec<P>::C* __restrict__ stage,
                                        int32_t* __restrict__ slots) {
  using C = typename Prec<P>::C;
  using Stager = WaveRecordStager<C, cap_stride(Lat::Q)>;
  static_assert(BS == NBR_BLOCK, "a work-group covers one pull-table block");
  const int64_t xr = blk * BS + threadIdx.x;
  const bool valid = xr < x1;
  // lanes past the end recompute the last element (in bounds, same block)
  // and store nothing; the record staging needs every lane of the wave
  const int64_t x = valid ? xr : x1 - 1;
  C g[Lat::Q];
  {
    int32_t j[Lat::Q];
    pull_sources_wg<Lat>(a, blk, (uint32_t)x, j, slots);
    gather_from<Lat, P>(src, x, a, j, g);
  }
  C drho, rho, u[3];
  // F32: moments and equilibria in FP64, the relaxation in FP32.  With all
  // of it in FP32 the rounding of the moment sums and equilibria dominated
  // the FP32 variant's error on fine meshes near tau = 1/2 (unused in the
  // other precisions; F16S is bound by its storage instead).
  double drho_w = 0, rho_w = 0, u_w[3] = {0, 0, 0}, uu_w = 0;
  if constexpr (P == MLBM_F32) {
    macro_g_wide<Lat>(g, (double)a.rho0, drho_w, rho_w, u_w);
    uu_w = dot_uu<Lat, double>(u_w);
    drho = (C)drho_w;
    rho = (C)rho_w;
#pragma unroll
    for (int b = 0; b < 3; ++b) u[b] = (C)u_w[b];
  } else {
    macro_g<Lat, C>(g, a.rho0, drho, rho, u);
  }
  const C uu = dot_uu<Lat, C>(u);
  auto post = [&](int i) -> C {
    if constexpr (P == MLBM_F32)
      return g[i] + a.omega * ((C)geq_i<Lat, double>(i, drho_w, rho_w, u_w, uu_w) - g[i]);
    else
      return g[i] + a.omega * (geq_i<Lat, C>(i, drho, rho, u, uu) - g[i]);
  };
  // interpolation sources keep their pre-collision moments
  const bool is_src = valid && x >= a.cap_begin && x < a.n_fluid;
  const uint64_t m = __ballot(is_src);
  if (m) {   // wave-uniform
    const int lane = threadIdx.x & 63;
    Stager w{stage + (threadIdx.x >> 6) * Stager::LDS_PER_WAVE, cap, (xr - lane) - a.cap_begin,
             m, lane, {}};
    record_values<Lat, C>(w, g, drho, rho, u, uu, a.omega);
  }
  using S = typename Prec<P>::S;
  bool ok = true;
  // Stores.  A whole work-group (all but the last of the range) puts its
  // post-collision values into an LDS tile [Q][BS] and writes each row's BS
  // consecutive values with aligned 16-byte stores: rows start on 128-byte
  // lines (padded row stride) and blk * BS is a multiple of 8, so the
  // vector memory instructions for the stores drop from Q per wave to about
  // Q * BS * sizeof(S) / (16 * BS) per thread.  The record stager's LDS is
  // the tile once every wave has finished its records.
  if (P != MLBM_F64 && (blk + 1) * BS <= x1) {
    __syncthreads();
    S* __restrict__ tile = reinterpret_cast<S*>(stage);
    const int t = threadIdx.x;
    if constexpr (P == MLBM_F16S) {
      ok = store_f16s_conserving<Lat>([&](int i, __half h) { tile[i * BS + t] = h; }, a, g,
                                      drho, rho, u, uu);
    } else {
#pragma unroll
      for (int i = 0; i < Lat::Q; ++i) tile[i * BS + t] = (S)post(i);   // FP32: the deviation
    }
    __syncthreads();
    typedef int VT __attribute__((ext_vector_type(4)));
    constexpr int PER = 16 / (int)sizeof(S);          // values per 16-byte chunk
    constexpr int CPR = BS / PER;                     // chunks per row
    const VT* __restrict__ tv = reinterpret_cast<const VT*>(tile);
    for (int c = t; c < Lat::Q * CPR; c += BS) {
      const int i = c / CPR, k = c % CPR;
      *reinterpret_cast<VT*>(dst + (int64_t)i * a.n + blk * BS + k * PER) = tv[c];
    }
  } else {
    if (!valid) return;
    if constexpr (P == MLBM_F16S) {
      ok = store_f16s_conserving<Lat>(
          [&](int i, __half h) { store_elem(dst + (int64_t)i * a.n, a.n, (uint32_t)x, h); }, a, g,
          drho, rho, u, uu);
    } else {
#pragma unroll
      for (int i = 0; i < Lat::Q; ++i)
        ok &= store_row<P>(dst + (int64_t)i * a.n, a.n, (uint32_t)x, post(i),
                           a.wr[Lat::wclass(i)], a.scale);
    }
  }
  const bool finite = (rho == rho) && (rho - rho == C(0));
  if (!finite || !ok)
    atomicOr(status, (finite ? 0u : (uint32_t)MLBM_STATUS_NONFINITE) |
                         (ok ? 0u : (uint32_t)MLBM_STATUS_F16_OVERFLOW));
}

template <class C, int Q>
constexpr int sc_stage_values(int bs) {
  return (bs / 64) * WaveRecordStager<C, cap_stride(Q)>::LDS_PER_WAVE;
}
// LDS of a stream-collide work-group, in compute values: the record stager,
// which is also the store tile of Q * bs stored values (not for FP64)
template <int P, int Q>
constexpr int sc_lds_values(int bs) {
  using C = typename Prec<P>::C;
  using S = typename Prec<P>::S;
  constexpr int tile = P == MLBM_F64 ? 0 : (int)((Q * 256 * sizeof(S) + sizeof(C) - 1) / sizeof(C));
  const int stage = sc_stage_values<C, Q>(bs);
  return stage > tile * bs / 256 ? stage : tile * bs / 256;
}

// One level's stream-collide over [0, x1); the block map balances the plain
// range and the tail (capture sources, inner ghosts) over the XCDs.
template <class Lat, int P, int BS>
__global__ __launch_bounds__(BS, (P == MLBM_F32 && Lat::Q == 19) ? 6 : 1) void k_stream_collide(
    const typename Prec<P>::S* __restrict__ src, typename Prec<P>::S* __restrict__ dst,
    int64_t x1, const LevelArgs<typename Prec<P>::C, Lat::Q> a,
    typename Prec<P>::C* __restrict__ cap, uint32_t* __restrict__ status) {
  using C = typename Prec<P>::C;
  __shared__ __align__(16) C stage[sc_lds_values<P, Lat::Q>(BS)];
  __shared__ int32_t slots[NBR_SLOTS];
  const int64_t blk = xcd_block2(blockIdx.x, gridDim.x, a.cap_begin / BS);
  sc_body<Lat, P, BS>(blk, x1, src, dst, a, cap, status, stage, slots);
}

// Stream-collides of several levels in one launch.  Consecutive
// stream-collides of different levels in the schedule touch disjoint data
// (each reads and writes only its own level), so they can run as one grid:
// segment s holds work-groups [first[s], first[s] + nb[s]); every segment
// starts at a multiple of 8 (on XCD 0), so it keeps the XCD-sliced block map
// of a launch of its own, and the few work-groups between segments exit.
constexpr int SC_MAX_SEG = 6;
template <class C, class S, int Q>
struct ScMulti {
  int nseg;
  int64_t first[SC_MAX_SEG];
  int64_t b0[SC_MAX_SEG];     // first pull-table block of the segment
  int64_t nb[SC_MAX_SEG];
  int64_t n_act[SC_MAX_SEG];
  const S* src[SC_MAX_SEG];
  S* dst[SC_MAX_SEG];
  C* cap[SC_MAX_SEG];
  LevelArgs<C, Q> a[SC_MAX_SEG];
};

template <class Lat, int P, int BS>
__global__ __launch_bounds__(BS, (P == MLBM_F32 && Lat::Q == 19) ? 6 : 1) void k_stream_collide_multi(
    const ScMulti<typename Prec<P>::C, typename Prec<P>::S, Lat::Q> m,
    uint32_t* __restrict__ status) {
  using C = typename Prec<P>::C;
  __shared__ __align__(16) C stage[sc_lds_values<P, Lat::Q>(BS)];
  __shared__ int32_t slots[NBR_SLOTS];
  int sg = 0;
  while (sg + 1 < m.nseg && (int64_t)blockIdx.x >= m.first[sg + 1]) ++sg;
  const int64_t b = (int64_t)blockIdx.x - m.first[sg];
  if (b >= m.nb[sg]) return;
  const LevelArgs<C, Lat::Q>& a = m.a[sg];
  const int64_t plain = a.cap_begin / BS - m.b0[sg];
  const int64_t blk = m.b0[sg] + xcd_block2(b, m.nb[sg], plain > 0 ? plain : 0);
  sc_body<Lat, P, BS>(blk, m.n_act[sg], m.src[sg], m.dst[sg], a, m.cap[sg], status, stage,
                      slots);
}

// --------------------------------------------------- interpolation --------
// A record view: drho, u, S, g^neq.
template <class Lat, class C>
struct Rec {
  const C* p;
  __device__ C drho() const { return p[cap_rho(Lat::Q)]; }
  __device__ C u(int a) const { return p[cap_u(Lat::Q) + a]; }
  __device__ C S(int k) const { return p[cap_s(Lat::Q) + k]; }
  __device__ C fneq(int i) const { return p[cap_fneq(Lat::Q) + i]; }
};

// A capture record read into registers with 16-byte loads (records start at
// multiples of their 64-byte-or-more stride; the loads stay inside it).
template <class Lat, class C>
struct RecV {
  static constexpr int V = 16 / (int)sizeof(C);
  static constexpr int N = (cap_used(Lat::Q) + V - 1) / V;
  static_assert(N * V <= cap_stride(Lat::Q), "record loads stay in the record");
  typedef C VT __attribute__((ext_vector_type(16 / sizeof(C))));
  C v[N * V];
  __device__ __forceinline__ void load(const C* __restrict__ p) {
    const VT* q = reinterpret_cast<const VT*>(p);
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const VT t = q[k];
#pragma unroll
      for (int e = 0; e < V; ++e) v[k * V + e] = t[e];
    }
  }
  __device__ C drho() const { return v[cap_rho(Lat::Q)]; }
  __device__ C u(int a) const { return v[cap_u(Lat::Q) + a]; }
  __device__ C S(int k) const { return v[cap_s(Lat::Q) + k]; }
  __device__ C fneq(int i) const { return v[cap_fneq(Lat::Q) + i]; }
};

// Writes the interpolated ghost: g* = g_eq(rho, u) + (1 - omega_t) g^neq
// into the pdf array; optionally its pre-collision record.
template <class Lat, int P>
__device__ __forceinline__ bool emit_ghost(typename Prec<P>::S* __restrict__ pdf, int64_t x,
                                           const LevelArgs<typename Prec<P>::C, Lat::Q>& a,
                                           typename Prec<P>::C drho, const typename Prec<P>::C* u,
                                           const typename Prec<P>::C* fneq) {
  using C = typename Prec<P>::C;
  const C rho = a.rho0 + drho;
  const C uu = dot_uu<Lat, C>(u);
  bool ok = true;
#pragma unroll
  for (int i = 0; i < Lat::Q; ++i) {
    const C gs = geq_i<Lat, C>(i, drho, rho, u, uu) + (C(1) - a.omega) * fneq[i];
    ok &= store_g<P>(pdf, (int64_t)i * a.n + x, gs, a.wr[Lat::wclass(i)], a.scale);
  }
  return ok;
}

// GhostFromFiner (Sec. 2.2, Steps 1-5) of coarse level: sources are the four
// fine children (0,0,0), (1,1,0), (1,0,1), (0,1,1) (2D: all four) read from
// the fine capture buffer; target is the parent's centre.  Closed form of
// the compact interpolation at the tetrahedron's centroid:
// u = mean(u_k) - 1/4 (a_xx + a_yy + a_zz) per component.
// gff_values gives the ghost's pre-collision drho, u and g^neq (rescaled to
// the coarse level) from the capture slots s[4] of its four fine sources.
// Velocity and density deviation are taken to coarse lattice units by
// `us` and `rs` (1 under acoustic scaling, where both are level invariant).
template <class Lat, class C>
__device__ __forceinline__ void gff_values(const int32_t* s, const C* __restrict__ cap_fine,
                                           C fneq_scale, C us, C rs, C& drho, C* u, C* fneq) {
  constexpr int D = Lat::D;
  RecV<Lat, C> r[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) r[k].load(cap_fine + (int64_t)s[k] * cap_stride(Lat::Q));
  u[0] = u[1] = u[2] = C(0);
  drho = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    drho += r[k].drho();
#pragma unroll
    for (int b = 0; b < D; ++b) u[b] += r[k].u(b);
  }
  drho *= C(0.25);
#pragma unroll
  for (int b = 0; b < D; ++b) u[b] *= C(0.25);
  if constexpr (D == 3) {
    // D_x = (-H + K + M - N)/2, D_y = (-H + K - M + N)/2, D_z = (-H - K + M + N)/2
    auto Dx = [&](int k) { return C(0.5) * (-r[0].S(k) + r[1].S(k) + r[2].S(k) - r[3].S(k)); };
    auto Dy = [&](int k) { return C(0.5) * (-r[0].S(k) + r[1].S(k) - r[2].S(k) + r[3].S(k)); };
    auto Dz = [&](int k) { return C(0.5) * (-r[0].S(k) - r[1].S(k) + r[2].S(k) + r[3].S(k)); };
    // S order: xx, yy, zz, xy, yz, xz
    const C axx = C(0.5) * Dx(0), axy = Dy(0), axz = Dz(0);
    const C bxy = Dx(1), byy = C(0.5) * Dy(1), byz = Dz(1);
    const C cxz = Dx(2), cyz = Dy(2), czz = C(0.5) * Dz(2);
    const C bxx = Dx(3) - C(0.5) * axy, ayy = Dy(3) - C(0.5) * bxy;
    const C cyy = Dy(4) - C(0.5) * byz, bzz = Dz(4) - C(0.5) * cyz;
    const C cxx = Dx(5) - C(0.5) * axz, azz = Dz(5) - C(0.5) * cxz;
    u[0] -= C(0.25) * (axx + ayy + azz);
    u[1] -= C(0.25) * (bxx + byy + bzz);
    u[2] -= C(0.25) * (cxx + cyy + czz);
  } else {
    // children (0,0), (1,0), (0,1), (1,1): D_x = (-P00 + P10 - P01 + P11)/2
    auto Dx = [&](int k) { return C(0.5) * (-r[0].S(k) + r[1].S(k) - r[2].S(k) + r[3].S(k)); };
    auto Dy = [&](int k) { return C(0.5) * (-r[0].S(k) - r[1].S(k) + r[2].S(k) + r[3].S(k)); };
    // S order: xx, yy, xy
    const C axx = C(0.5) * Dx(0), axy = Dy(0);
    const C bxy = Dx(1), byy = C(0.5) * Dy(1);
    const C bxx = Dx(2) - C(0.5) * axy, ayy = Dy(2) - C(0.5) * bxy;
    u[0] -= C(0.25) * (axx + ayy);
    u[1] -= C(0.25) * (bxx + byy);
  }
  drho *= rs;
#pragma unroll
  for (int b = 0; b < D; ++b) u[b] *= us;
#pragma unroll
  for (int i = 0; i < Lat::Q; ++i)
    fneq[i] = C(0.25) * (r[0].fneq(i) + r[1].fneq(i) + r[2].fneq(i) + r[3].fneq(i)) * fneq_scale;
}

// Capture-record values of an interpolated ghost, in slot order, handed to
// a writer (the S of the record uses the target level's omega).
template <class Lat, class C, class Wr>
__device__ __forceinline__ void ghost_record(Wr& w, C drho, const C* u, const C* fneq, C omega,
                                             C rho0) {
  constexpr int D = Lat::D;
  const C rho = rho0 + drho;
#pragma unroll
  for (int i = 0; i < Lat::Q; ++i) w.put(cap_fneq(Lat::Q) + i, fneq[i]);
  w.put(cap_rho(Lat::Q), drho);
#pragma unroll
  for (int b = 0; b < D; ++b) w.put(cap_u(Lat::Q) + b, u[b]);
  const C pref = -C(1.5) * omega / rho;
#pragma unroll
  for (int k = 0; k < Lat::NS; ++k) {
    const int aa = strain_a(D, k), bb = strain_b(D, k);
    C s = 0;
#pragma unroll
    for (int i = 0; i < Lat::Q; ++i) {
      const int cc = Lat::c(i, aa) * Lat::c(i, bb);
      if (cc > 0) s += fneq[i];
      if (cc < 0) s -= fneq[i];
    }
    w.put(cap_s(Lat::Q) + k, pref * s);
  }
  w.finish(cap_used(Lat::Q));
}

// Plain writer into an LDS row (no padding stores).
template <class C>
struct RowWriter {
  C* p;
  __device__ __forceinline__ void put(int c, C v) { p[c] = v; }
  __device__ __forceinline__ void finish(int) {}
};

// One GhostFromFiner ghost j: pdfs and capture record.
template <class Lat, int P>
__device__ __forceinline__ void gff_ghost(
    int64_t j, typename Prec<P>::S* __restrict__ pdf, int64_t gff_begin, int64_t n_gff,
    const int32_t* __restrict__ slots, const typename Prec<P>::C* __restrict__ cap_fine,
    typename Prec<P>::C* __restrict__ cap_coarse, int64_t cap_gff_begin,
    const LevelArgs<typename Prec<P>::C, Lat::Q>& a, typename Prec<P>::C fneq_scale,
    typename Prec<P>::C us, typename Prec<P>::C rs, uint32_t* __restrict__ status) {
  using C = typename Prec<P>::C;
  C drho, u[3], fneq[Lat::Q];
  int32_t s[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) s[k] = slots[k * n_gff + j];
  gff_values<Lat, C>(s, cap_fine, fneq_scale, us, rs, drho, u, fneq);
  const bool ok = emit_ghost<Lat, P>(pdf, gff_begin + j, a, drho, u, fneq);
  // pre-collision record of the ghost: it is a GhostFromCoarser source
  RecordWriter<C> w{cap_coarse + (cap_gff_begin + j) * cap_stride(Lat::Q), {}};
  ghost_record<Lat, C>(w, drho, u, fneq, a.omega, a.rho0);
  if (!ok) atomicOr(status, (uint32_t)MLBM_STATUS_F16_OVERFLOW);
}

template <class Lat, int P>
__global__ __launch_bounds__(64) void k_fill_gff(
    typename Prec<P>::S* __restrict__ pdf, int64_t gff_begin, int64_t n_gff,
    const int32_t* __restrict__ slots, const typename Prec<P>::C* __restrict__ cap_fine,
    typename Prec<P>::C* __restrict__ cap_coarse, int64_t cap_gff_begin,
    const LevelArgs<typename Prec<P>::C, Lat::Q> a, typename Prec<P>::C fneq_scale,
    typename Prec<P>::C us, typename Prec<P>::C rs, uint32_t* __restrict__ status) {
  const int64_t j = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (j >= n_gff) return;
  gff_ghost<Lat, P>(j, pdf, gff_begin, n_gff, slots, cap_fine, cap_coarse, cap_gff_begin, a,
                    fneq_scale, us, rs, status);
}

// GhostFromCoarser (Sec. 2.2) of fine level, both layers.  One work-group
// takes GPB parent groups; the capture records of each parent's
// neighbourhood (13 cells in 3D, 9 in 2D) are staged in LDS and shared by
// the parent's children.  For child octant s the sources are
// H = P, K = P + (s_x, s_y, 0), M = P + (s_x, 0, s_z), N = P + (0, s_y, s_z)
// (2D: P, P + s_x, P + s_y, P + s_x + s_y); target at s/4.
// Coarse GhostFromFiner records computed in place of being read, for a
// GhostFromCoarser fill that runs in the same launch as the GhostFromFiner
// fill producing them.  With `tab` set the staging reads the group table's
// int4 rows (see LevelPlan::grp_tab): {slot, -, -, -} for a record read from
// memory, {-2 - f0, f1, f2, f3} for one formed from the fine records f0..f3
// (one load fewer on that path), {-1, -, -, -} for an absent cell.
template <class C>
struct GffOnTheFly {
  const int4* tab = nullptr;
  const C* cap_fine = nullptr;
  C fneq_scale = 0, omega = 0, rho0 = 0;
  C us = 1, rs = 1;   // fine -> coarse velocity and density-deviation units
};

template <int Q> constexpr int gfc_lds_stride() { return cap_used(Q) | 1; }  // odd: no conflicts
template <int D> constexpr int gfc_groups_per_block() { return 64 / group_children(D); }

template <class Lat, int P>
__device__ __forceinline__ void gfc_groups(
    int64_t blk, typename Prec<P>::C* __restrict__ sh, typename Prec<P>::S* __restrict__ pdf,
    int64_t n_groups, const int32_t* __restrict__ grp_src, const int32_t* __restrict__ grp_child,
    const typename Prec<P>::C* __restrict__ cap_coarse,
    const LevelArgs<typename Prec<P>::C, Lat::Q>& a, typename Prec<P>::C fneq_scale,
    typename Prec<P>::C us, typename Prec<P>::C rs,
    const GffOnTheFly<typename Prec<P>::C>& fly, uint32_t* __restrict__ status) {
  using C = typename Prec<P>::C;
  constexpr int D = Lat::D;
  constexpr int NB = group_slots(D), NC = group_children(D);
  constexpr int GPB = gfc_groups_per_block<D>();
  constexpr int ST = cap_stride(Lat::Q);
  constexpr int USED = cap_used(Lat::Q);            // components actually read
  constexpr int LST = gfc_lds_stride<Lat::Q>();
  const int64_t g0 = blk * GPB;
  // one record per thread and pass: a single slot lookup, contiguous reads
  for (int r = threadIdx.x; r < GPB * NB; r += 64) {
    const int gl = r / NB, sl = r % NB;
    const int64_t g = g0 + gl;
    int4 t = {-1, 0, 0, 0};
    if (g < n_groups) {
      if (fly.tab)
        t = fly.tab[(int64_t)sl * n_groups + g];
      else
        t.x = grp_src[(int64_t)sl * n_groups + g];
    }
    const int32_t slot = t.x;
    C* dst = sh + r * LST;
    if (slot <= -2) {
      C drho, u[3], fneq[Lat::Q];
      const int32_t fs[4] = {-2 - t.x, t.y, t.z, t.w};
      gff_values<Lat, C>(fs, fly.cap_fine, fly.fneq_scale, fly.us, fly.rs, drho, u, fneq);
      RowWriter<C> w{dst};
      ghost_record<Lat, C>(w, drho, u, fneq, fly.omega, fly.rho0);
    } else if (slot >= 0) {
      RecV<Lat, C> src;
      src.load(cap_coarse + (int64_t)slot * ST);
#pragma unroll
      for (int c = 0; c < USED; ++c) dst[c] = src.v[c];
    } else {
#pragma unroll
      for (int c = 0; c < USED; ++c) dst[c] = C(0);
    }
  }
  __syncthreads();
  const int gl = threadIdx.x / NC, c = threadIdx.x % NC;
  const int64_t g = g0 + gl;
  if (g >= n_groups) return;
  const int32_t target = grp_child[(int64_t)c * n_groups + g];
  if (target < 0) return;
  const int sx = (c & 1) ? 1 : -1, sy = (c & 2) ? 1 : -1, sz = (c & 4) ? 1 : -1;
  const C* base = sh + gl * NB * LST;
  C u[3] = {0, 0, 0}, drho, fneq[Lat::Q];
  if constexpr (D == 3) {
    const Rec<Lat, C> H{base + group_slot_of(3, 0, 0, 0) * LST};
    const Rec<Lat, C> K{base + group_slot_of(3, sx, sy, 0) * LST};
    const Rec<Lat, C> M{base + group_slot_of(3, sx, 0, sz) * LST};
    const Rec<Lat, C> N{base + group_slot_of(3, 0, sy, sz) * LST};
    const C hx = C(0.5) * sx, hy = C(0.5) * sy, hz = C(0.5) * sz;
    auto Dx = [&](int k) { return hx * (-H.S(k) + K.S(k) + M.S(k) - N.S(k)); };
    auto Dy = [&](int k) { return hy * (-H.S(k) + K.S(k) - M.S(k) + N.S(k)); };
    auto Dz = [&](int k) { return hz * (-H.S(k) - K.S(k) + M.S(k) + N.S(k)); };
    const C axx = C(0.5) * Dx(0), axy = Dy(0), axz = Dz(0);
    const C bxy = Dx(1), byy = C(0.5) * Dy(1), byz = Dz(1);
    const C cxz = Dx(2), cyz = Dy(2), czz = C(0.5) * Dz(2);
    const C bxx = Dx(3) - C(0.5) * axy, ayy = Dy(3) - C(0.5) * bxy;
    const C cyy = Dy(4) - C(0.5) * byz, bzz = Dz(4) - C(0.5) * cyz;
    const C cxx = Dx(5) - C(0.5) * axz, azz = Dz(5) - C(0.5) * cxz;
    const C T = Dz(3) + Dx(4) + Dy(5);
    const C ayz = T - C(2) * Dx(4), bxz = T - C(2) * Dy(5), cxy = T - C(2) * Dz(3);
    const C sxy = C(sx * sy), syz = C(sy * sz), sxz = C(sx * sz);
    const C w5 = C(0.625), w1 = C(0.125);
#pragma unroll
    for (int b = 0; b < 3; ++b) u[b] = w5 * H.u(b) + w1 * (K.u(b) + M.u(b) + N.u(b));
    u[0] -= C(3.0 / 16.0) * (axx + ayy + azz) + C(1.0 / 16.0) * (sxy * axy + syz * ayz + sxz * axz);
    u[1] -= C(3.0 / 16.0) * (bxx + byy + bzz) + C(1.0 / 16.0) * (sxy * bxy + syz * byz + sxz * bxz);
    u[2] -= C(3.0 / 16.0) * (cxx + cyy + czz) + C(1.0 / 16.0) * (sxy * cxy + syz * cyz + sxz * cxz);
    drho = w5 * H.drho() + w1 * (K.drho() + M.drho() + N.drho());
#pragma unroll
    for (int i = 0; i < Lat::Q; ++i)
      fneq[i] = (w5 * H.fneq(i) + w1 * (K.fneq(i) + M.fneq(i) + N.fneq(i))) * fneq_scale;
  } else {
    const Rec<Lat, C> R0{base + group_slot_of(2, 0, 0, 0) * LST};
    const Rec<Lat, C> Rx{base + group_slot_of(2, sx, 0, 0) * LST};
    const Rec<Lat, C> Ry{base + group_slot_of(2, 0, sy, 0) * LST};
    const Rec<Lat, C> Rxy{base + group_slot_of(2, sx, sy, 0) * LST};
    const C hx = C(0.5) * sx, hy = C(0.5) * sy;
    auto Dx = [&](int k) { return hx * (-R0.S(k) + Rx.S(k) - Ry.S(k) + Rxy.S(k)); };
    auto Dy = [&](int k) { return hy * (-R0.S(k) - Rx.S(k) + Ry.S(k) + Rxy.S(k)); };
    const C axx = C(0.5) * Dx(0), axy = Dy(0);
    const C bxy = Dx(1), byy = C(0.5) * Dy(1);
    const C bxx = Dx(2) - C(0.5) * axy, ayy = Dy(2) - C(0.5) * bxy;
    const C w9 = C(9.0 / 16.0), w3 = C(3.0 / 16.0), w1 = C(1.0 / 16.0);
#pragma unroll
    for (int b = 0; b < 2; ++b) u[b] = w9 * R0.u(b) + w3 * (Rx.u(b) + Ry.u(b)) + w1 * Rxy.u(b);
    u[0] -= C(3.0 / 16.0) * (axx + ayy);
    u[1] -= C(3.0 / 16.0) * (bxx + byy);
    drho = w9 * R0.drho() + w3 * (Rx.drho() + Ry.drho()) + w1 * Rxy.drho();
#pragma unroll
    for (int i = 0; i < Lat::Q; ++i)
      fneq[i] = (w9 * R0.fneq(i) + w3 * (Rx.fneq(i) + Ry.fneq(i)) + w1 * Rxy.fneq(i)) * fneq_scale;
  }
  // to fine lattice units (1 under acoustic scaling)
  drho *= rs;
#pragma unroll
  for (int b = 0; b < D; ++b) u[b] *= us;
  if (!emit_ghost<Lat, P>(pdf, target, a, drho, u, fneq))
    atomicOr(status, (uint32_t)MLBM_STATUS_F16_OVERFLOW);
}

template <class Lat, int P>
__global__ __launch_bounds__(64) void k_fill_gfc(
    typename Prec<P>::S* __restrict__ pdf, int64_t n_groups,
    const int32_t* __restrict__ grp_src, const int32_t* __restrict__ grp_child,
    const typename Prec<P>::C* __restrict__ cap_coarse,
    const LevelArgs<typename Prec<P>::C, Lat::Q> a, typename Prec<P>::C fneq_scale,
    typename Prec<P>::C us, typename Prec<P>::C rs, uint32_t* __restrict__ status) {
  using C = typename Prec<P>::C;
  constexpr int D = Lat::D;
  __shared__ C sh[gfc_groups_per_block<D>() * group_slots(D) * gfc_lds_stride<Lat::Q>()];
  gfc_groups<Lat, P>(blockIdx.x, sh, pdf, n_groups, grp_src, grp_child, cap_coarse, a, fneq_scale,
                     us, rs, GffOnTheFly<C>{}, status);
}

// The fills of one synchronisation of levels (k, k+1), for one or several
// level pairs (segments) per launch.  In a segment, work-groups
// [0, nb_gff) fill the GhostFromFiner ghosts of level k (pdfs and records),
// the rest the GhostFromCoarser ghosts of level k+1, which compute the
// coarse GhostFromFiner records they read from the fine records instead of
// waiting for them (same results as k_fill_gff then k_fill_gfc).
// Consecutive fills of the schedule, fill(k+1) then fill(k), touch disjoint
// data: each writes the GhostFromFiner ghosts and records of its coarse
// level and the GhostFromCoarser ghosts of its fine level, and reads only
// fluid capture records.
constexpr int FILL_MAX_SEG = 4;
template <class C, class S, int Q>
struct FillSeg {
  int64_t first, nb_gff, nb;     // work-groups [first, first + nb); GFF part first
  S* pdf_c;
  int64_t gff_begin, n_gff;
  const int32_t* gff_slot;
  const C* cap_fine;
  C* cap_coarse;
  int64_t cap_gff_begin;
  LevelArgs<C, Q> ac;
  C scale_gff, us_gff, rs_gff;   // g^neq rescale, velocity and density units
  S* pdf_f;
  int64_t n_groups;
  const int32_t* grp_src;
  const int4* grp_tab;
  const int32_t* grp_child;
  LevelArgs<C, Q> af;
  C scale_gfc, us_gfc, rs_gfc;
};
template <class C, class S, int Q>
struct FillMulti {
  int nseg;
  FillSeg<C, S, Q> seg[FILL_MAX_SEG];
};

template <class Lat, int P>
__global__ __launch_bounds__(64) void k_fill_sync(
    const FillMulti<typename Prec<P>::C, typename Prec<P>::S, Lat::Q> m,
    uint32_t* __restrict__ status) {
  using C = typename Prec<P>::C;
  constexpr int D = Lat::D;
  __shared__ C sh[gfc_groups_per_block<D>() * group_slots(D) * gfc_lds_stride<Lat::Q>()];
  int sg = 0;
  while (sg + 1 < m.nseg && (int64_t)blockIdx.x >= m.seg[sg + 1].first) ++sg;
  const auto& f = m.seg[sg];
  const int64_t b = (int64_t)blockIdx.x - f.first;
  if (b >= f.nb) return;
  if (b < f.nb_gff) {
    const int64_t j = b * 64 + threadIdx.x;
    if (j < f.n_gff)
      gff_ghost<Lat, P>(j, f.pdf_c, f.gff_begin, f.n_gff, f.gff_slot, f.cap_fine, f.cap_coarse,
                        f.cap_gff_begin, f.ac, f.scale_gff, f.us_gff, f.rs_gff, status);
    return;
  }
  GffOnTheFly<C> fly;
  fly.tab = f.grp_tab;
  fly.cap_fine = f.cap_fine;
  fly.fneq_scale = f.scale_gff;
  fly.omega = f.ac.omega;
  fly.rho0 = f.ac.rho0;
  fly.us = f.us_gff;
  fly.rs = f.rs_gff;
  gfc_groups<Lat, P>(b - f.nb_gff, sh, f.pdf_f, f.n_groups, f.grp_src, f.grp_child,
                     (const C*)f.cap_coarse, f.af, f.scale_gfc, f.us_gfc, f.rs_gfc, fly, status);
}

// -------------------------------------------------------------- init ------
// f = f^eq(rho, u) + f^neq(S) with f^neq_i = -(w_i rho/(cs^2 omega)) Q_i:S,
// computed in FP64 and returned as g = f - w rho0.
template <class Lat>
__device__ __forceinline__ void init_g(const double* __restrict__ rho_in,
                                       const double* __restrict__ u_in,
                                       const double* __restrict__ S_in, int64_t nf, int64_t x,
                                       double rho0, double omega, double* g) {
  const double rho = rho_in[x];
  double u[3] = {0, 0, 0}, S[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int a = 0; a < Lat::D; ++a) u[a] = u_in[(int64_t)a * nf + x];
  if (S_in) {
#pragma unroll
    for (int k = 0; k < Lat::NS; ++k) S[k] = S_in[(int64_t)k * nf + x];
  }
  const double uu = dot_uu<Lat, double>(u);
  double trS = 0;
#pragma unroll
  for (int a = 0; a < Lat::D; ++a) trS += S[a];
#pragma unroll
  for (int i = 0; i < Lat::Q; ++i) {
    double cu = 0, cSc = 0;
#pragma unroll
    for (int a = 0; a < Lat::D; ++a) cu += Lat::c(i, a) * u[a];
#pragma unroll
    for (int k = 0; k < Lat::NS; ++k) {
      const int aa = strain_a(Lat::D, k), bb = strain_b(Lat::D, k);
      cSc += (aa == bb ? 1.0 : 2.0) * Lat::c(i, aa) * Lat::c(i, bb) * S[k];
    }
    const double w = Lat::w(i);
    const double feq = w * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    const double QS = cSc - trS / 3.0;
    const double fneq = -(w * rho / (omega / 3.0)) * QS;
    g[i] = feq + fneq - w * rho0;
  }
}

template <class Lat, int P>
__global__ __launch_bounds__(256) void k_init(const double* __restrict__ rho_in,
                                              const double* __restrict__ u_in,
                                              const double* __restrict__ S_in, int64_t nf,
                                              typename Prec<P>::S* __restrict__ pdf,
                                              const LevelArgs<typename Prec<P>::C, Lat::Q> a,
                                              double rho0, double omega) {
  const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (x >= nf) return;
  double g[Lat::Q];
  init_g<Lat>(rho_in, u_in, S_in, nf, x, rho0, omega, g);
  double drho, rho, u[3];
  macro_g<Lat, double>(g, rho0, drho, rho, u);
  const double uu = dot_uu<Lat, double>(u);
#pragma unroll
  for (int i = 0; i < Lat::Q; ++i) {
    const double gs = g[i] + omega * (geq_i<Lat, double>(i, drho, rho, u, uu) - g[i]);
    store_g<P>(pdf, (int64_t)i * a.n + x, (typename Prec<P>::C)gs, a.wr[Lat::wclass(i)], a.scale);
  }
}

// Ghost entries [nf, n) of a pdf array set to the rest state w_i rho0 (a
// zero deviation).  Stream-collides that update inner ghost layers beyond
// what the fluid reads (diffusive scaling) may read ghost entries of the
// array that no fill writes; they then hold finite values.
template <class Lat, int P>
__global__ __launch_bounds__(256) void k_rest_ghosts(typename Prec<P>::S* __restrict__ pdf,
                                                     int64_t nf, int64_t n,
                                                     const LevelArgs<typename Prec<P>::C, Lat::Q> a) {
  const int64_t x = nf + (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (x >= n) return;
#pragma unroll
  for (int i = 0; i < Lat::Q; ++i)
    store_g<P>(pdf, (int64_t)i * a.n + x, typename Prec<P>::C(0), a.wr[Lat::wclass(i)], a.scale);
}

template <class Lat, int P>
__global__ __launch_bounds__(256) void k_init_capture(
    const double* __restrict__ rho_in, const double* __restrict__ u_in,
    const double* __restrict__ S_in, int64_t nf, const int32_t* __restrict__ cap_elem,
    int64_t n_cap, typename Prec<P>::C* __restrict__ cap, double rho0, double omega) {
  const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s >= n_cap) return;
  double g[Lat::Q];
  init_g<Lat>(rho_in, u_in, S_in, nf, cap_elem[s], rho0, omega, g);
  write_record<Lat, double>(cap + s * cap_stride(Lat::Q), g, rho0, omega);
}

// Max |f - w rho0| over the initial state of a level (FP16 scale choice).
template <class Lat>
__global__ __launch_bounds__(256) void k_init_maxdev(const double* __restrict__ rho_in,
                                                     const double* __restrict__ u_in,
                                                     const double* __restrict__ S_in, int64_t nf,
                                                     double rho0, double omega,
                                                     double* __restrict__ partial) {
  __shared__ double sm[256];
  double m = 0;
  for (int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x; x < nf;
       x += (int64_t)gridDim.x * 256) {
    double g[Lat::Q];
    init_g<Lat>(rho_in, u_in, S_in, nf, x, rho0, omega, g);
#pragma unroll
    for (int i = 0; i < Lat::Q; ++i) m = fmax(m, fabs(g[i]));
  }
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sm[0];
}

// --------------------------------------------------------- state I/O ------
// pdf rows have stride a.n (the padded row stride), out rows stride n
template <class Lat, int P>
__global__ __launch_bounds__(256) void k_get_pdf(const typename Prec<P>::S* __restrict__ pdf,
                                                 int64_t n, const LevelArgs<typename Prec<P>::C, Lat::Q> a,
                                                 double* __restrict__ out) {
  const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (x >= n) return;
#pragma unroll
  for (int i = 0; i < Lat::Q; ++i)
    out[(int64_t)i * n + x] = (double)a.wr[Lat::wclass(i)] + (double)load_g<P>(pdf, (int64_t)i * a.n + x, a.wr[Lat::wclass(i)], a.inv_scale);
}

template <class Lat, int P>
__global__ __launch_bounds__(256) void k_set_pdf(typename Prec<P>::S* __restrict__ pdf, int64_t n,
                                                 const LevelArgs<typename Prec<P>::C, Lat::Q> a,
                                                 const double* __restrict__ in) {
  const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (x >= n) return;
#pragma unroll
  for (int i = 0; i < Lat::Q; ++i)
    store_g<P>(pdf, (int64_t)i * a.n + x, (typename Prec<P>::C)(in[(int64_t)i * n + x] - (double)a.wr[Lat::wclass(i)]),
               a.wr[Lat::wclass(i)], a.scale);
}

template <class Lat, int P>
__global__ __launch_bounds__(256) void k_get_moments(const typename Prec<P>::S* __restrict__ pdf,
                                                     int64_t nf,
                                                     const LevelArgs<typename Prec<P>::C, Lat::Q> a,
                                                     double* __restrict__ out) {
  const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (x >= nf) return;
  double g[Lat::Q];
#pragma unroll
  for (int i = 0; i < Lat::Q; ++i) g[i] = (double)load_g<P>(pdf, (int64_t)i * a.n + x, a.wr[Lat::wclass(i)], a.inv_scale);
  double drho, rho, u[3];
  macro_g<Lat, double>(g, (double)a.rho0, drho, rho, u);
  out[x] = rho;
#pragma unroll
  for (int b = 0; b < Lat::D; ++b) out[(int64_t)(1 + b) * nf + x] = u[b];
}

// Pre-collision state of the fluid elements as the level's last
// stream-collide gathered it.  A pull scheme keeps the array that
// stream-collide read (the post-collision state one level substep earlier,
// wall-link values included): the fills that follow write only the ghosts
// of the other array.  Pulling from it again, with the same table decode and
// boundary rules, gives the gathered values exactly.  WHAT 0: the pdfs
// f = w rho0 + g, FP64 [Q][nf].  WHAT 1: the strain rate of Sec. 2.1,
// S_ab = -(3 omega / (2 rho)) sum_i c_ia c_ib f^neq_i with f^neq = f - f^eq
// of the gathered f, formed in FP64 with the exact lattice weights, FP64
// [NS][nf] in the order xx, yy, zz, xy, yz, xz (2D: xx, yy, xy).  One
// work-group per pull-table block; the blocks of [0, nf) are whole or the
// last one is cut, whose surplus threads take part in the slot staging only.
template <class Lat, int P, int WHAT>
__global__ __launch_bounds__(256) void k_get_pulled(
    const typename Prec<P>::S* __restrict__ prev, int64_t nf,
    const LevelArgs<typename Prec<P>::C, Lat::Q> a, double omega, double* __restrict__ out) {
  using C = typename Prec<P>::C;
  static_assert(NBR_BLOCK == 256, "a work-group covers one pull-table block");
  __shared__ int32_t slots[NBR_SLOTS];
  const int64_t blk = blockIdx.x;
  const int64_t xr = blk * 256 + threadIdx.x;
  const int64_t x = xr < nf ? xr : nf - 1;
  C g[Lat::Q];
  {
    int32_t j[Lat::Q];
    pull_sources_wg<Lat>(a, blk, (uint32_t)x, j, slots);
    gather_from<Lat, P>(prev, x, a, j, g);
  }
  if (xr >= nf) return;
  if constexpr (WHAT == 0) {
#pragma unroll
    for (int i = 0; i < Lat::Q; ++i)
      out[(int64_t)i * nf + x] = (double)a.wr[Lat::wclass(i)] + (double)g[i];
  } else {
    constexpr int D = Lat::D;
    double gd[Lat::Q];   // f - w with the exact weights
#pragma unroll
    for (int i = 0; i < Lat::Q; ++i)
      gd[i] = ((double)a.wr[Lat::wclass(i)] + (double)g[i]) - Lat::w(i);
    double drho, rho, u[3];
    macro_g<Lat, double>(gd, 1.0, drho, rho, u);
    const double uu = dot_uu<Lat, double>(u);
    double pi[Lat::NS];
#pragma unroll
    for (int k = 0; k < Lat::NS; ++k) pi[k] = 0.0;
#pragma unroll
    for (int i = 0; i < Lat::Q; ++i) {
      const double fneq = gd[i] - geq_i<Lat, double>(i, drho, rho, u, uu);
#pragma unroll
      for (int k = 0; k < Lat::NS; ++k) {
        const int cc = Lat::c(i, strain_a(D, k)) * Lat::c(i, strain_b(D, k));
        if (cc > 0) pi[k] += fneq;
        if (cc < 0) pi[k] -= fneq;
      }
    }
    const double pref = -1.5 * omega / rho;
#pragma unroll
    for (int k = 0; k < Lat::NS; ++k) out[(int64_t)k * nf + x] = pref * pi[k];
  }
}

// Given pre-collision pdfs of the fluid elements (FP64 [Q][nf]), stores
// their BGK post-collision values (Eq. bgk) as the level's state and the
// pre-collision moments of the interpolation sources as their capture
// records: what a stream-collide does once it has gathered f.
template <class Lat, int P>
__global__ __launch_bounds__(256) void k_set_pre(typename Prec<P>::S* __restrict__ pdf, int64_t nf,
                                                 const LevelArgs<typename Prec<P>::C, Lat::Q> a,
                                                 const double* __restrict__ in,
                                                 typename Prec<P>::C* __restrict__ cap,
                                                 uint32_t* __restrict__ status) {
  using C = typename Prec<P>::C;
  const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (x >= nf) return;
  C g[Lat::Q];
#pragma unroll
  for (int i = 0; i < Lat::Q; ++i)
    g[i] = (C)(in[(int64_t)i * nf + x] - (double)a.wr[Lat::wclass(i)]);
  C drho, rho, u[3];
  macro_g<Lat, C>(g, a.rho0, drho, rho, u);
  const C uu = dot_uu<Lat, C>(u);
  if (x >= a.cap_begin)
    write_record_m<Lat, C, C>(cap + (x - a.cap_begin) * cap_stride(Lat::Q), g, drho, rho, u, uu,
                              a.omega);
  bool ok = true;
  if constexpr (P == MLBM_F16S) {
    ok = store_f16s_conserving<Lat>(
        [&](int i, __half h) { store_elem(pdf + (int64_t)i * a.n, a.n, (uint32_t)x, h); }, a, g,
        drho, rho, u, uu);
  } else {
#pragma unroll
    for (int i = 0; i < Lat::Q; ++i) {
      const C gs = g[i] + a.omega * (geq_i<Lat, C>(i, drho, rho, u, uu) - g[i]);
      ok &= store_row<P>(pdf + (int64_t)i * a.n, a.n, (uint32_t)x, gs, a.wr[Lat::wclass(i)],
                         a.scale);
    }
  }
  const bool finite = (rho == rho) && (rho - rho == C(0));
  if (!finite || !ok)
    atomicOr(status, (finite ? 0u : (uint32_t)MLBM_STATUS_NONFINITE) |
                         (ok ? 0u : (uint32_t)MLBM_STATUS_F16_OVERFLOW));
}

// ------------------------------------------------------- diagnostics ------
// Per-block FP64 partial sums (deterministic tree in LDS).  Mass is summed
// as deviations drho; the host-side constant rho0 * n_fluid is added in the
// final pass.
constexpr int DIAG_BLOCKS = 512;
constexpr int DIAG_VALS = 5;  // drho, ke, fx, fy, fz

__device__ __forceinline__ void block_sum(double* sm, double v, double* out) {
  sm[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sm[0];
  __syncthreads();
}

template <class Lat, int P>
__global__ __launch_bounds__(256) void k_diag_partial(
    const typename Prec<P>::S* __restrict__ pdf, int64_t nf, const int32_t* __restrict__ bounce,
    int64_t n_bounce, const LevelArgs<typename Prec<P>::C, Lat::Q> a, double* __restrict__ partial) {
  __shared__ double sm[256];
  double m = 0, ke = 0, F[3] = {0, 0, 0};
  for (int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x; x < nf;
       x += (int64_t)gridDim.x * 256) {
    double g[Lat::Q];
#pragma unroll
    for (int i = 0; i < Lat::Q; ++i) g[i] = (double)load_g<P>(pdf, (int64_t)i * a.n + x, a.wr[Lat::wclass(i)], a.inv_scale);
    double drho, rho, u[3];
    macro_g<Lat, double>(g, (double)a.rho0, drho, rho, u);
    m += drho;
    ke += 0.5 * rho * dot_uu<Lat, double>(u);
  }
  // momentum exchange with halfway bounce-back: 2 c_i f*_i(x) for each link
  // whose pull source x - c_j is solid, i = opp(j) pointing into the solid
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n_bounce;
       t += (int64_t)gridDim.x * 256) {
    const int64_t x = bounce[t];
    const int j = bounce[n_bounce + t];
    const int i = Lat::opp(j);
    const double f = (double)a.wr[Lat::wclass(i)] + (double)load_g<P>(pdf, (int64_t)i * a.n + x, a.wr[Lat::wclass(i)], a.inv_scale);
#pragma unroll
    for (int b = 0; b < Lat::D; ++b) F[b] += 2.0 * Lat::c(i, b) * f;
  }
  // links with a wall fraction: their returning value replaces f*_i(x) in
  // c_i (f*_i(x) + f_j(x, t+1)), i = opp(j) (same rule as the stream-collide)
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < a.n_wall;
       t += (int64_t)gridDim.x * 256) {
    const int4 w = a.wall[t];
    if (w.x < 0) continue;   // padding
    const int j = w.y;
    const int i = (j & 1) ? j + 1 : j - 1;
    const double wr = (double)wall_weight<Lat, typename Prec<P>::C>(a, w.w);
    auto f_at = [&](int dir, int64_t e) {
      return wr + (double)load_g<P>(pdf, (int64_t)dir * a.n + e, (typename Prec<P>::C)wr,
                                    a.inv_scale);
    };
    const double fo = f_at(i, w.x), q = a.wall_q[t];
    double v = fo;
    if (q < 0.5) {
      if (w.z >= 0) v = 2.0 * q * fo + (1.0 - 2.0 * q) * f_at(i, w.z);
    } else {
      v = fo / (2.0 * q) + (1.0 - 1.0 / (2.0 * q)) * f_at(j, w.x);
    }
#pragma unroll
    for (int k = 1; k < Lat::Q; ++k)
      if (k == i) {
#pragma unroll
        for (int b = 0; b < Lat::D; ++b) F[b] += Lat::c(k, b) * (v - fo);
      }
  }
  double* out = partial + (int64_t)blockIdx.x * DIAG_VALS;
  block_sum(sm, m, out + 0);
  block_sum(sm, ke, out + 1);
  block_sum(sm, F[0], out + 2);
  block_sum(sm, F[1], out + 3);
  block_sum(sm, F[2], out + 4);
}

struct DiagLevel {
  double vol, force_scale, rho0_nf;
  double unit2;   // (level-L0 velocity per level-L velocity)^2
};

// Final pass: one block; levels summed coarse to fine in fixed order.
static __global__ __launch_bounds__(256) void k_diag_final(const double* __restrict__ partial, int nlev,
                                                     const DiagLevel* __restrict__ lv, uint32_t mask,
                                                     int d, double* __restrict__ out) {
  __shared__ double sm[256];
  __shared__ double tot[DIAG_VALS];
  if (threadIdx.x < DIAG_VALS) tot[threadIdx.x] = 0;
  __syncthreads();
  for (int k = 0; k < nlev; ++k) {
    for (int v = 0; v < DIAG_VALS; ++v) {
      double s = 0;
      for (int b = threadIdx.x; b < DIAG_BLOCKS; b += 256)
        s += partial[((int64_t)k * DIAG_BLOCKS + b) * DIAG_VALS + v];
      double r;
      block_sum(sm, s, &sm[0]);
      if (threadIdx.x == 0) {
        r = sm[0];
        if (v == 0) tot[0] += lv[k].vol * (lv[k].rho0_nf + r * lv[k].unit2);
        else if (v == 1) tot[1] += lv[k].vol * r * lv[k].unit2;
        else tot[v] += lv[k].force_scale * r;
      }
      __syncthreads();
    }
  }
  if (threadIdx.x == 0) {
    int o = 0;
    if (mask & MLBM_DIAG_MASS) out[o++] = tot[0];
    if (mask & MLBM_DIAG_KE) out[o++] = tot[1];
    if (mask & MLBM_DIAG_FORCE)
      for (int b = 0; b < d; ++b) out[o++] = tot[2 + b];
  }
}

}  // namespace mlbm
