// Host-side plan: level-wise element lists and index tables.
#pragma once

#include <cstdint>
#include <vector>

#include "common.hpp"

namespace mlbm {

struct LevelPlan {
  int level = 0;
  int64_t n = 0, n_fluid = 0, n_inner = 0, n_outer = 0, n_gff = 0;
  int64_t cap_begin = 0;           // fluid [cap_begin, n_fluid) are sources
  std::vector<uint64_t> tid;       // [n]
  std::vector<int32_t> coords;     // [d][n]
  std::vector<int32_t> nbr;        // [q-1][n]
  std::vector<int32_t> gfc_src;    // [4][n_gfc] element indices on L-1
  std::vector<int32_t> gff_src;    // [4][n_gff] element indices on L+1
  std::vector<int32_t> cap_elem;   // [n_cap_fluid] capture sources (fluid)
  std::vector<int32_t> gff_slot;   // [4][n_gff] capture slots on L+1
  int64_t n_groups = 0;            // GhostFromCoarser parent groups
  std::vector<int32_t> grp_src;    // [slots][n_groups] capture slots on L-1
  // [slots][n_groups][4]: the synchronous fill's staging rows.  A slot whose
  // L-1 record is a GhostFromFiner ghost's (formed on the fly from the L
  // records) holds {-2 - f0, f1, f2, f3}, the capture slots on L of that
  // ghost's four sources; other slots {grp_src, 0, 0, 0}.
  std::vector<int32_t> grp_tab;
  std::vector<int32_t> grp_child;  // [children][n_groups] element idx on L
  std::vector<int32_t> bounce;     // [2][n_bounce] (element, direction)
  // links with a wall fraction (linear interpolated bounce-back), sorted by
  // element then pull direction: [n_wall][4] {x, j, x2, weight class of j},
  // and their fractions; the device copy is padded with links {-1, 0, -1, 0}
  // so that no element's links straddle a chunk of NBR_BLOCK links
  std::vector<int32_t> wall;
  std::vector<double> wall_q;
  std::vector<int32_t> wall_dev;
  std::vector<double> wall_dev_q;
  // transpose of the wall pre-pass in gather form: the entries it reads or
  // writes [n_ent][4] {direction, element, keep own value (not written), 0},
  // per entry its terms [ptr[e], ptr[e+1]) with the written entry they come
  // from [nnz][2] {direction, element}, the coefficient and the x-drag seed
  // coefficient c_ox (coefficient - [the entry is the link's own])
  std::vector<int32_t> wadj_ent, wadj_ptr, wadj_src;
  std::vector<double> wadj_coef, wadj_seed;

  // The pull table as the device holds it, over the updated range in blocks
  // of NBR_BLOCK elements: per (block, direction) up to NBR_BASES base
  // indices and per entry a 16-bit code (base << 14 | offset from it), or
  // 0xFFFC..0xFFFF for the link codes -4..-1.  A block whose neighbours
  // need more bases is "wide": nhdr[b][2] = w marks it, its code rows hold
  // the low 16 bits of the int32 entries and row block w of nbr_wide the
  // high 16 bits.  A direction whose sources in the block are the Morton
  // neighbours of the elements shifted by at most two constants (runs of
  // the treeID order split at one Morton threshold) reads no codes: its
  // bit is set in nhdr[b][0] and its slot holds {k0, k1, t0, t1}.
  std::vector<uint16_t> nbr16;     // [q-1][n_nbr_blocks * NBR_BLOCK]
  std::vector<int32_t> nbase;      // [n_nbr_blocks][q-1][NBR_BASES]
  std::vector<uint16_t> nbr_wide;  // [q-1][n_wide * NBR_BLOCK]
  std::vector<int32_t> nhdr;       // [n_nbr_blocks][NBR_HDR]
  bool morton = false;             // some blocks hold Morton directions
  int64_t n_wide = 0;

  // adjoint tables
  std::vector<int32_t> unassigned[2];  // [2][cnt] (element, direction) fluid-range
                                       // entries no pull reads; variant 0: fluid
                                       // updated, 1: fluid and inner ghosts
  std::vector<int32_t> copy_elems;     // updated elements with a COPY link
  std::vector<int32_t> csr_ptr;        // [n_cap(L-1)+1] coarse slot -> contributions
  std::vector<int32_t> csr_ent;        // group * group_slots + neighbourhood slot

  int64_t n_gfc() const { return n_inner + n_outer; }
  int64_t n_active_max() const { return n_fluid + n_inner; }
  int64_t n_nbr_blocks() const { return (n_active_max() + NBR_BLOCK - 1) / NBR_BLOCK; }
  int64_t n_cap_fluid() const { return (int64_t)cap_elem.size(); }
  int64_t n_cap() const { return n_cap_fluid() + n_gff; }
  int64_t n_bounce() const { return (int64_t)bounce.size() / 2; }
  int64_t n_wall() const { return (int64_t)wall_q.size(); }
  int64_t n_wall_dev() const { return (int64_t)wall_dev_q.size(); }
  int64_t n_wadj() const { return (int64_t)wadj_ptr.size() - (wadj_ptr.empty() ? 0 : 1); }
};

}  // namespace mlbm

struct mlbm_plan {
  int stencil = 0, d = 0, q = 0, level0 = 0;
  int gfc_layers = 2;   // GhostFromCoarser layers: 2 acoustic, 4 diffusive scaling
  int32_t origin[3] = {0, 0, 0}, extent[3] = {1, 1, 1};
  int32_t faces[6] = {0, 0, 0, 0, 0, 0};
  std::vector<mlbm::LevelPlan> lv;
  int nlev() const { return (int)lv.size(); }
};
