// Internal definitions shared by the host plan builder and the HIP kernels.
#pragma once

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/mlbm.h"

#if defined(__HIPCC__)
#define MLBM_HD __host__ __device__
#else
#define MLBM_HD
#endif

namespace mlbm {

// Velocity sets (Sec. 2.1).  Direction 0 is at rest; directions 2k-1 and 2k
// are opposite, so opp(i) = i + 1 for odd i and i - 1 for even i > 0.
// cs^2 = 1/3; weights give an isotropic fourth moment.
struct D2Q9 {
  static constexpr int D = 2, Q = 9, STENCIL = MLBM_D2Q9;
  static constexpr int NS = 3;  // strain components xx, yy, xy
  MLBM_HD static constexpr int c(int i, int a) {
    constexpr int t[9][2] = {{0, 0}, {1, 0}, {-1, 0}, {0, 1}, {0, -1},
                             {1, 1}, {-1, -1}, {1, -1}, {-1, 1}};
    return t[i][a];
  }
  MLBM_HD static constexpr double w(int i) {
    return i == 0 ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
  }
  // weight class: 0 rest, 1 axis, 2 diagonal
  MLBM_HD static constexpr int wclass(int i) { return i == 0 ? 0 : (i <= 4 ? 1 : 2); }
  MLBM_HD static constexpr int opp(int i) {
    return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1);
  }
};

struct D3Q19 {
  static constexpr int D = 3, Q = 19, STENCIL = MLBM_D3Q19;
  static constexpr int NS = 6;  // strain components xx, yy, zz, xy, yz, xz
  MLBM_HD static constexpr int c(int i, int a) {
    constexpr int t[19][3] = {
        {0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},
        {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
        {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
        {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
    return t[i][a];
  }
  MLBM_HD static constexpr double w(int i) {
    return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
  }
  // weight class: 0 rest, 1 axis, 2 diagonal
  MLBM_HD static constexpr int wclass(int i) { return i == 0 ? 0 : (i <= 6 ? 1 : 2); }
  MLBM_HD static constexpr int opp(int i) {
    return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1);
  }
};

// D3Q27: rest, 6 axis, 12 edge (as D3Q19), 8 corner directions; opposite
// directions sit in rows 2k-1, 2k.
struct D3Q27 {
  static constexpr int D = 3, Q = 27, STENCIL = MLBM_D3Q27;
  static constexpr int NS = 6;
  MLBM_HD static constexpr int c(int i, int a) {
    constexpr int t[27][3] = {
        {0, 0, 0},   {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},   {0, -1, 0},  {0, 0, 1},
        {0, 0, -1},  {1, 1, 0},   {-1, -1, 0}, {1, -1, 0},  {-1, 1, 0},  {1, 0, 1},
        {-1, 0, -1}, {1, 0, -1},  {-1, 0, 1},  {0, 1, 1},   {0, -1, -1}, {0, 1, -1},
        {0, -1, 1},  {1, 1, 1},   {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1}, {1, -1, 1},
        {-1, 1, -1}, {-1, 1, 1},  {1, -1, -1}};
    return t[i][a];
  }
  MLBM_HD static constexpr double w(int i) {
    return i == 0 ? 8.0 / 27.0 : (i <= 6 ? 2.0 / 27.0 : (i <= 18 ? 1.0 / 54.0 : 1.0 / 216.0));
  }
  // weight class: 0 rest, 1 axis, 2 edge, 3 corner
  MLBM_HD static constexpr int wclass(int i) { return i == 0 ? 0 : (i <= 6 ? 1 : (i <= 18 ? 2 : 3)); }
  MLBM_HD static constexpr int opp(int i) {
    return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1);
  }
};

// Strain component order (a, b) for NS components.
MLBM_HD constexpr int strain_a(int d, int k) {
  return d == 3 ? (k == 0 ? 0 : k == 1 ? 1 : k == 2 ? 2 : k == 3 ? 0 : k == 4 ? 1 : 0)
                : (k == 0 ? 0 : k == 1 ? 1 : 0);
}
MLBM_HD constexpr int strain_b(int d, int k) {
  return d == 3 ? (k == 0 ? 0 : k == 1 ? 1 : k == 2 ? 2 : k == 3 ? 1 : k == 4 ? 2 : 2)
                : (k == 0 ? 0 : k == 1 ? 1 : 1);
}

inline int stencil_q(int stencil) {
  return stencil == MLBM_D2Q9 ? 9 : (stencil == MLBM_D3Q27 ? 27 : 19);
}
// Lattice constants by stencil for host code.
inline int stencil_c(int stencil, int i, int a) {
  return stencil == MLBM_D2Q9 ? D2Q9::c(i, a)
                              : (stencil == MLBM_D3Q27 ? D3Q27::c(i, a) : D3Q19::c(i, a));
}
inline double stencil_w(int stencil, int i) {
  return stencil == MLBM_D2Q9 ? D2Q9::w(i) : (stencil == MLBM_D3Q27 ? D3Q27::w(i) : D3Q19::w(i));
}
inline int stencil_wclass(int stencil, int i) {
  return stencil == MLBM_D2Q9 ? D2Q9::wclass(i)
                              : (stencil == MLBM_D3Q27 ? D3Q27::wclass(i) : D3Q19::wclass(i));
}
inline int stencil_opp(int stencil, int i) {
  return stencil == MLBM_D2Q9 ? D2Q9::opp(i) : (stencil == MLBM_D3Q27 ? D3Q27::opp(i) : D3Q19::opp(i));
}
inline int stencil_d(int stencil) { return stencil == MLBM_D2Q9 ? 2 : 3; }

// Opposite directions carry equal weights (true of every symmetric lattice).
template <class Lat>
MLBM_HD constexpr bool opposite_weights_equal() {
  for (int i = 0; i < Lat::Q; ++i)
    if (Lat::w(i) != Lat::w(Lat::opp(i))) return false;
  return true;
}

// Compressed pull table (see LevelPlan): block size, bases per block and
// direction, largest offset from a base, first code value.
constexpr int NBR_BLOCK = 256;
constexpr int NBR_BASES = 4;
constexpr int NBR_SPAN = 16380;
constexpr uint32_t NBR_CODE0 = 0xFFFCu;
// Per-block header of the pull table: mask of directions whose sources
// follow from Morton arithmetic, Morton code minus index of the block's
// elements (mod 2^32), wide row block (-1: none), unused.
constexpr int NBR_HDR = 4;
// offset past every code row: a lane that needs no code loads from here and
// gets 0 from the buffer range check, without a memory access
constexpr uint32_t NBR_NO_CODE = 0x7FFFFFF8u;
// Default policy for Morton directions (mlbm_set_morton_policy): a block
// takes them only if at least NBR_MIN_MORTON qualify (a block mixing both
// kinds decodes both readings), and a level only if at least
// NBR_LEVEL_MIN_MORTON of its (block, direction) pairs would (a level with
// Morton directions reads each block's header before its codes; with the
// slots staged in LDS that wait measures as nothing, so every level may).
constexpr int NBR_MIN_MORTON = 6;
constexpr double NBR_LEVEL_MIN_MORTON = 0.0;

// Level-local Morton code (treeID minus the level's first ID; bit b of axis
// a at position d*b + a), kept to its low 32 bits.  Moving one cell along an
// axis adds or subtracts the axis's lowest bit with the carry passed through
// the other axes' bits (dilated integer arithmetic); modulo 2^32 this gives
// the low 32 bits of the exact code.
template <int D>
MLBM_HD constexpr uint32_t morton_axis_bits(int a) {
  return D == 3 ? (a == 0 ? 0x49249249u : (a == 1 ? 0x92492492u : 0x24924924u))
                : (a == 0 ? 0x55555555u : 0xAAAAAAAAu);
}
template <int D>
MLBM_HD inline uint32_t morton_step(uint32_t m, int a, int s) {
  const uint32_t mask = morton_axis_bits<D>(a), one = 1u << a;
  const uint32_t t = s > 0 ? (m | ~mask) + one : (m & mask) - one;
  return (t & mask) | (m & ~mask);
}
// Morton code of the cell the pull of direction i reads: x - c_i.
template <class Lat>
MLBM_HD inline uint32_t morton_pull(uint32_t m, int i) {
  for (int a = 0; a < Lat::D; ++a)
    if (Lat::c(i, a) != 0) m = morton_step<Lat::D>(m, a, -Lat::c(i, a));
  return m;
}

// Work-group order.  Consecutive work-groups of a launch go to the 8 XCDs in
// turn (dispatch position b runs on XCD b mod 8), and each XCD has its own
// L2.  xcd_block maps dispatch position b of nb to a logical block so that
// every XCD streams one contiguous slice of the range.
MLBM_HD inline int64_t xcd_block(int64_t b, int64_t nb) {
  const int64_t q = nb >> 3, r = nb & 7, xcd = b & 7, k = b >> 3;
  return xcd * q + (xcd < r ? xcd : r) + k;
}

// Two-range variant: logical blocks [0, nb1) (plain fluid) and [nb1, nb)
// (capture sources and ghosts, which do more work per element) are each
// split into contiguous per-XCD slices.  Every XCD runs its share of the
// heavier tail first, so the slow blocks overlap the streaming of the plain
// ones instead of trailing behind them.  A bijection of [0, nb) for any
// 0 <= nb1 <= nb.
MLBM_HD inline int64_t xcd_block2(int64_t b, int64_t nb, int64_t nb1) {
  const int64_t x = b & 7, k = b >> 3;
  const int64_t q = nb >> 3, r = nb & 7, q1 = nb1 >> 3, r1 = nb1 & 7;
  const int64_t cnt = q + (x < r ? 1 : 0);          // positions on XCD x
  const int64_t cnt1 = q1 + (x < r1 ? 1 : 0);       // its plain blocks
  const int64_t cnt2 = cnt - cnt1;                  // its tail blocks
  if (k < cnt2) return nb1 + x * (q - q1) + (x < r ? x : r) - (x < r1 ? x : r1) + k;
  return x * q1 + (x < r1 ? x : r1) + (k - cnt2);
}

// Capture record: f^neq (q), drho, u (d), S (NS), padded to 16, 32 or 48
// values for D2Q9, D3Q19, D3Q27 (a multiple of the record stager's 64-byte
// phase; D3Q19 FP32: one 128-byte line).  f^neq and drho come first so that
// the q+1 values formed in the collide loop fill whole 16-byte chunks.
MLBM_HD constexpr int cap_dim(int q) { return q == 9 ? 2 : 3; }
MLBM_HD constexpr int cap_stride(int q) { return q == 27 ? 48 : (q == 19 ? 32 : 16); }
MLBM_HD constexpr int cap_fneq(int) { return 0; }
MLBM_HD constexpr int cap_rho(int q) { return q; }
MLBM_HD constexpr int cap_u(int q) { return cap_rho(q) + 1; }
MLBM_HD constexpr int cap_s(int q) { return cap_u(q) + cap_dim(q); }
MLBM_HD constexpr int cap_used(int q) { return cap_s(q) + (cap_dim(q) == 3 ? 6 : 3); }

// Neighbourhood slots of a GhostFromCoarser parent group: 3D uses the
// parent and its 12 edge neighbours, 2D the parent and its 8 neighbours.
MLBM_HD constexpr int group_slots(int d) { return d == 3 ? 13 : 9; }
MLBM_HD constexpr int group_children(int d) { return d == 3 ? 8 : 4; }
// slot index of offset (ox, oy[, oz]) in {-1,0,1}; -1 if not a slot.
MLBM_HD constexpr int group_slot_of(int d, int ox, int oy, int oz) {
  if (d == 2) return (ox + 1) + 3 * (oy + 1);  // 0..8, parent = 4
  // 3D: parent = 0; edges (two non-zero components) = 1..12
  if (ox == 0 && oy == 0 && oz == 0) return 0;
  if (oz == 0 && ox != 0 && oy != 0) return 1 + ((ox > 0) ? 0 : 2) + ((oy > 0) ? 0 : 1);
  if (oy == 0 && ox != 0 && oz != 0) return 5 + ((ox > 0) ? 0 : 2) + ((oz > 0) ? 0 : 1);
  if (ox == 0 && oy != 0 && oz != 0) return 9 + ((oy > 0) ? 0 : 2) + ((oz > 0) ? 0 : 1);
  return -1;
}
MLBM_HD constexpr int group_parent_slot(int d) { return d == 3 ? 0 : 4; }

// thread-local error reporting
void set_error(const char* fmt, ...);
int32_t fail(int32_t code, const char* fmt, ...);

}  // namespace mlbm
