// Host plan builder: decodes leaf treeIDs (Sec. 3.1), classifies ghost
// elements (Sec. 2.2), lays out the level-wise element lists (Sec. 3.2) and
// builds the neighbour, interpolation-source and capture tables that the
// device kernels consume.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdlib>
#include <cstdarg>
#include <cstring>
#include <memory>
#include <new>
#include <numeric>
#include <stdexcept>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "plan.hpp"

namespace mlbm {

static thread_local std::string g_last_error;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
}

int32_t fail(int32_t code, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

namespace {

constexpr int32_t V_EMPTY = -1, V_SOLID = -2, V_REFINED = -3, V_GFF = -4,
                  V_GFC_IN = -5, V_GFC_OUT = -6;

struct MeshError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

uint64_t level_first_id(int L, int d) {
  uint64_t s = 0;
  for (int k = 0; k < L; ++k) s += (uint64_t)1 << (d * k);
  return s;
}

uint64_t morton(const int64_t* c, int d, int L) {
  uint64_t m = 0;
  for (int b = 0; b < L; ++b)
    for (int a = 0; a < d; ++a) m |= (uint64_t)((c[a] >> b) & 1) << (d * b + a);
  return m;
}

struct Geom {
  int d = 3, level0 = 0;
  int64_t o[3] = {0, 0, 0}, e[3] = {1, 1, 1};
  bool per[3] = {false, false, false};
  int faces[6] = {0, 0, 0, 0, 0, 0};
  int64_t lo(int a, int L) const { return o[a] << (L - level0); }
  int64_t hi(int a, int L) const { return (o[a] + e[a]) << (L - level0); }
  // wraps periodic axes in place; returns a bit mask of crossed faces
  int wrap(int64_t* c, int L) const {
    int out = 0;
    for (int a = 0; a < d; ++a) {
      const int64_t l = lo(a, L), h = hi(a, L);
      if (per[a]) {
        const int64_t ext = h - l;
        int64_t r = (c[a] - l) % ext;
        if (r < 0) r += ext;
        c[a] = l + r;
      } else if (c[a] < l) {
        out |= 1 << (2 * a);
      } else if (c[a] >= h) {
        out |= 1 << (2 * a + 1);
      }
    }
    return out;
  }
  int32_t face_code(int crossed) const {
    bool eq = false, cp = false;
    for (int f = 0; f < 2 * d; ++f) {
      if (!(crossed & (1 << f))) continue;
      eq |= faces[f] == MLBM_FACE_EQ;
      cp |= faces[f] == MLBM_FACE_COPY;
    }
    return eq ? MLBM_NBR_EQ : (cp ? MLBM_NBR_COPY : MLBM_NBR_BOUNCE);
  }
};

// Position -> value map of one level: a dense grid over the level's
// bounding region when that is compact, a hash map otherwise.
struct CellMap {
  int d = 3, L = 0;
  int64_t lo[3] = {0, 0, 0}, ext[3] = {1, 1, 1};
  bool dense = true;
  std::vector<int32_t> grid;
  std::unordered_map<int64_t, int32_t> hm;

  bool in_box(const int64_t* c) const {
    for (int a = 0; a < d; ++a)
      if (c[a] < lo[a] || c[a] >= lo[a] + ext[a]) return false;
    return true;
  }
  int64_t dkey(const int64_t* c) const {
    int64_t k = 0;
    for (int a = d - 1; a >= 0; --a) k = k * ext[a] + (c[a] - lo[a]);
    return k;
  }
  int64_t skey(const int64_t* c) const {
    int64_t k = 0;
    for (int a = d - 1; a >= 0; --a) k = (k << L) | c[a];
    return k;
  }
  int32_t get(const int64_t* c) const {
    if (dense) return in_box(c) ? grid[dkey(c)] : V_EMPTY;
    auto it = hm.find(skey(c));
    return it == hm.end() ? V_EMPTY : it->second;
  }
  void set(const int64_t* c, int32_t v) {
    if (dense) {
      if (!in_box(c)) throw MeshError("internal: position outside level map");
      grid[dkey(c)] = v;
    } else {
      hm[skey(c)] = v;
    }
  }
};

struct LevelWork {
  std::vector<int64_t> fluid, solid;  // [count*d]
  int64_t bb_lo[3], bb_hi[3];
  bool bb_set = false;
  CellMap map;
  std::vector<int64_t> gff, gfc;      // provisional ghost coords
  std::vector<int64_t> refined;       // refined positions (coords)
  std::vector<int64_t> ring;          // fluid positions touching refined ones
  int64_t deeper = 0;
};

void extend_bb(LevelWork& w, const int64_t* c, int d) {
  if (!w.bb_set) {
    for (int a = 0; a < d; ++a) w.bb_lo[a] = w.bb_hi[a] = c[a];
    w.bb_set = true;
    return;
  }
  for (int a = 0; a < d; ++a) {
    w.bb_lo[a] = std::min(w.bb_lo[a], c[a]);
    w.bb_hi[a] = std::max(w.bb_hi[a], c[a]);
  }
}

template <class F>
void for_offsets(int d, int r, F&& fn) {
  int64_t o[3] = {0, 0, 0};
  const int side = 2 * r + 1;
  int total = 1;
  for (int a = 0; a < d; ++a) total *= side;
  for (int k = 0; k < total; ++k) {
    int t = k, dist = 0;
    for (int a = 0; a < d; ++a) {
      o[a] = (t % side) - r;
      t /= side;
      dist = std::max(dist, (int)std::llabs(o[a]));
    }
    if (dist) fn(o, dist);
  }
}

// Splits [0, n) into contiguous chunks over the hardware threads.
template <class F>
void parallel_for(int64_t n, F&& fn) {
  unsigned nt = std::thread::hardware_concurrency();
  nt = std::max(1u, std::min(nt, 16u));
  if (n < (1 << 16) || nt == 1) {
    fn((int64_t)0, n);
    return;
  }
  std::vector<std::thread> th;
  const int64_t chunk = (n + nt - 1) / nt;
  for (unsigned t = 0; t < nt; ++t) {
    const int64_t a = (int64_t)t * chunk, b = std::min(n, a + chunk);
    if (a < b) th.emplace_back([&fn, a, b] { fn(a, b); });
  }
  for (auto& t : th) t.join();
}

// Sorts v: contiguous chunks sorted on the hardware threads, then merged
// pairwise in parallel rounds.
template <class T>
void parallel_sort(std::vector<T>& v) {
  unsigned nt = std::thread::hardware_concurrency();
  nt = std::max(1u, std::min(nt, 16u));
  const int64_t n = (int64_t)v.size();
  if (n < (1 << 20) || nt == 1) {
    std::sort(v.begin(), v.end());
    return;
  }
  std::vector<int64_t> b(nt + 1);
  for (unsigned t = 0; t <= nt; ++t) b[t] = n * t / nt;
  {
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t)
      th.emplace_back([&v, &b, t] { std::sort(v.begin() + b[t], v.begin() + b[t + 1]); });
    for (auto& t : th) t.join();
  }
  for (unsigned w = 1; w < nt; w *= 2) {
    std::vector<std::thread> th;
    for (unsigned t = 0; t + w < nt; t += 2 * w) {
      const int64_t lo = b[t], mid = b[t + w], hi = b[std::min(t + 2 * w, nt)];
      th.emplace_back([&v, lo, mid, hi] {
        std::inplace_merge(v.begin() + lo, v.begin() + mid, v.begin() + hi);
      });
    }
    for (auto& t : th) t.join();
  }
}

struct PhaseTimer {
  bool on = std::getenv("MLBM_PLAN_TIMING") != nullptr;
  std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
  void mark(const char* what) {
    if (!on) return;
    auto n = std::chrono::steady_clock::now();
    fprintf(stderr, "[plan] %-28s %8.3f s\n", what, std::chrono::duration<double>(n - t).count());
    t = n;
  }
};

// Device form of the pull table (LevelPlan::nbr16 ...): per block and
// direction the distinct neighbour indices are grouped greedily in
// ascending order into runs shorter than NBR_SPAN, one base per run.
// Morton-direction policy for plans created from now on.
double g_morton_level_min = NBR_LEVEL_MIN_MORTON;
int g_morton_block_min = NBR_MIN_MORTON;
int g_gfc_layers = 2;

// Marks the (block, direction) pairs whose sources follow from Morton
// arithmetic: every element of the block has Morton code x + kself, and
// the sources of direction i are mo + k0 below the threshold t0 + t1 and
// mo + k1 from it, mo being the Morton code of x - c_i (all mod 2^32).
// A block keeps them if it has g_morton_block_min of them, the level only
// if they cover g_morton_level_min of its (block, direction) pairs.
template <class Lat>
void mark_morton_directions(LevelPlan& lp, uint64_t first, const std::vector<char>& wide) {
  constexpr int q = Lat::Q;
  const int64_t n = lp.n, act = lp.n_active_max(), nblk = lp.n_nbr_blocks();
  const int64_t ld = nblk * NBR_BLOCK;
  std::vector<uint32_t> regm((size_t)nblk, 0), kself((size_t)nblk, 0);
  std::vector<uint32_t> slot((size_t)nblk * (q - 1) * 4, 0);
  parallel_for(nblk, [&](int64_t b0, int64_t b1) {
    std::pair<uint32_t, uint32_t> rk[NBR_BLOCK];
    uint32_t m[NBR_BLOCK];
    for (int64_t b = b0; b < b1; ++b) {
      if (wide[b]) continue;
      const int64_t x0 = b * NBR_BLOCK;
      const int cnt = (int)(std::min(act, x0 + NBR_BLOCK) - x0);
      const uint32_t ks = (uint32_t)(lp.tid[x0] - first) - (uint32_t)x0;
      bool same = true;
      for (int l = 0; l < cnt && same; ++l) {
        m[l] = (uint32_t)(lp.tid[x0 + l] - first);
        same = m[l] - (uint32_t)(x0 + l) == ks;
      }
      if (!same) continue;
      uint32_t rm = 0;
      uint32_t* sl = &slot[(size_t)b * (q - 1) * 4];
      for (int i = 1; i < q; ++i) {
        const int32_t* row = &lp.nbr[(size_t)(i - 1) * n + x0];
        bool ok = true;
        uint32_t t0 = 0xFFFFFFFFu;
        for (int l = 0; l < cnt && ok; ++l) {
          ok = row[l] >= 0;
          const uint32_t mo = morton_pull<Lat>(m[l], i);
          rk[l] = {mo, (uint32_t)row[l] - mo};
          t0 = std::min(t0, mo);
        }
        if (!ok) continue;
        for (int l = 0; l < cnt; ++l) rk[l].first -= t0;
        std::sort(rk, rk + cnt);
        if (rk[cnt - 1].first >= 0x80000000u) continue;
        const uint32_t k0 = rk[0].second;
        int l = 0;
        while (l < cnt && rk[l].second == k0) ++l;
        const uint32_t t1 = l < cnt ? rk[l].first : 0xFFFFFFFFu;
        const uint32_t k1 = l < cnt ? rk[l].second : k0;
        for (; l < cnt && ok; ++l) ok = rk[l].second == k1;
        if (!ok) continue;
        rm |= 1u << i;
        uint32_t* s4 = sl + (i - 1) * 4;
        s4[0] = k0;
        s4[1] = k1;
        s4[2] = t0;
        s4[3] = t1;
      }
      if (__builtin_popcount(rm) >= g_morton_block_min) {
        regm[b] = rm;
        kself[b] = ks;
      }
    }
  });
  int64_t pairs = 0;
  for (int64_t b = 0; b < nblk; ++b) pairs += __builtin_popcount(regm[b]);
  lp.morton = pairs > 0 && (double)pairs >= g_morton_level_min * (double)(nblk * (q - 1));
  if (!lp.morton) return;
  parallel_for(nblk, [&](int64_t b0, int64_t b1) {
    for (int64_t b = b0; b < b1; ++b) {
      if (!regm[b]) continue;
      const int64_t x0 = b * NBR_BLOCK;
      const int cnt = (int)(std::min(act, x0 + NBR_BLOCK) - x0);
      for (int i = 1; i < q; ++i) {
        if (!((regm[b] >> i) & 1u)) continue;
        int32_t* bb = &lp.nbase[((size_t)b * (q - 1) + (i - 1)) * NBR_BASES];
        const uint32_t* s4 = &slot[((size_t)b * (q - 1) + (i - 1)) * 4];
        for (int t = 0; t < 4; ++t) bb[t] = (int32_t)s4[t];
        for (int e = 0; e < cnt; ++e) lp.nbr16[(size_t)(i - 1) * ld + x0 + e] = 0;
      }
      lp.nhdr[(size_t)b * NBR_HDR + 0] = (int32_t)regm[b];
      lp.nhdr[(size_t)b * NBR_HDR + 1] = (int32_t)kself[b];
    }
  });
}

void compress_pull_table(LevelPlan& lp, int q, int d, uint64_t first) {
  const int64_t n = lp.n, act = lp.n_active_max(), nblk = lp.n_nbr_blocks();
  const int64_t ld = nblk * NBR_BLOCK;
  lp.nbr16.assign((size_t)(q - 1) * ld, (uint16_t)0xFFFFu);
  lp.nbase.assign((size_t)nblk * (q - 1) * NBR_BASES, 0);
  std::vector<char> wide((size_t)nblk, 0);
  parallel_for(nblk, [&](int64_t b0, int64_t b1) {
    int32_t vals[NBR_BLOCK];
    for (int64_t b = b0; b < b1; ++b) {
      const int64_t x0 = b * NBR_BLOCK, x1 = std::min(act, x0 + NBR_BLOCK);
      for (int i = 1; i < q && !wide[b]; ++i) {
        const int32_t* row = &lp.nbr[(size_t)(i - 1) * n];
        int cnt = 0;
        for (int64_t x = x0; x < x1; ++x)
          if (row[x] >= 0) vals[cnt++] = row[x];
        std::sort(vals, vals + cnt);
        int32_t base[NBR_BASES];
        int nb = 0;
        for (int t = 0; t < cnt; ++t)
          if (nb == 0 || vals[t] - base[nb - 1] >= NBR_SPAN) {
            if (nb == NBR_BASES) {
              wide[b] = 1;
              break;
            }
            base[nb++] = vals[t];
          }
        if (wide[b]) break;
        int32_t* bb = &lp.nbase[((size_t)b * (q - 1) + (i - 1)) * NBR_BASES];
        for (int t = 0; t < nb; ++t) bb[t] = base[t];
        uint16_t* out = &lp.nbr16[(size_t)(i - 1) * ld];
        for (int64_t x = x0; x < x1; ++x) {
          const int32_t v = row[x];
          if (v < 0) {
            out[x] = (uint16_t)(0x10000 + v);
            continue;
          }
          int t = nb - 1;
          while (base[t] > v) --t;   // the run holding v starts at the last base <= v
          out[x] = (uint16_t)(((uint32_t)t << 14) | (uint32_t)(v - base[t]));
        }
      }
    }
  });
  lp.n_wide = 0;
  const int64_t ld16 = ld;
  std::vector<int64_t> wide_blocks;
  for (int64_t b = 0; b < nblk; ++b)
    if (wide[b]) wide_blocks.push_back(b);
  lp.n_wide = (int64_t)wide_blocks.size();
  const int64_t ldw = lp.n_wide * NBR_BLOCK;
  lp.nbr_wide.assign((size_t)(q - 1) * ldw, (uint16_t)0xFFFFu);
  lp.nhdr.assign((size_t)nblk * NBR_HDR, 0);
  for (int64_t b = 0; b < nblk; ++b) lp.nhdr[(size_t)b * NBR_HDR + 2] = -1;
  for (int64_t w = 0; w < lp.n_wide; ++w) {
    const int64_t b = wide_blocks[w];
    int32_t* bb = &lp.nbase[(size_t)b * (q - 1) * NBR_BASES];
    for (int t = 0; t < (q - 1) * NBR_BASES; ++t) bb[t] = 0;
    lp.nhdr[(size_t)b * NBR_HDR + 2] = (int32_t)w;
    const int64_t x0 = b * NBR_BLOCK, x1 = std::min(act, x0 + NBR_BLOCK);
    for (int i = 1; i < q; ++i)
      for (int64_t x = x0; x < x1; ++x) {
        const uint32_t v = (uint32_t)lp.nbr[(size_t)(i - 1) * n + x];
        lp.nbr16[(size_t)(i - 1) * ld16 + x] = (uint16_t)(v & 0xFFFFu);
        lp.nbr_wide[(size_t)(i - 1) * ldw + (size_t)w * NBR_BLOCK + (x - x0)] = (uint16_t)(v >> 16);
      }
  }
  if (q == 27)
    mark_morton_directions<D3Q27>(lp, first, wide);
  else if (q == 19)
    mark_morton_directions<D3Q19>(lp, first, wide);
  else
    mark_morton_directions<D2Q9>(lp, first, wide);
}

void build_plan(mlbm_plan& P, const uint64_t* leaf_ids, int64_t n_leaves,
                const uint64_t* solid_ids, int64_t n_solids) {
  const int d = P.d, q = P.q;
  PhaseTimer T;
  Geom g;
  g.d = d;
  g.level0 = P.level0;
  for (int a = 0; a < d; ++a) {
    g.o[a] = P.origin[a];
    g.e[a] = P.extent[a];
    g.per[a] = P.faces[2 * a] == MLBM_FACE_PERIODIC;
  }
  for (int f = 0; f < 2 * d; ++f) g.faces[f] = P.faces[f];
  const int max_level = d == 3 ? 20 : 30;

  // ---- decode ------------------------------------------------------
  auto decode = [&](uint64_t t, int& L, int64_t* c) {
    L = 0;
    while (L < max_level && level_first_id(L + 1, d) <= t) ++L;
    if (L >= max_level) throw MeshError("treeID beyond the supported depth");
    uint64_t off = t - level_first_id(L, d);
    for (int a = 0; a < d; ++a) c[a] = 0;
    for (int b = 0; b < L; ++b)
      for (int a = 0; a < d; ++a) c[a] |= (int64_t)((off >> (d * b + a)) & 1) << b;
  };
  std::vector<int> lvl_leaf(n_leaves), lvl_solid(n_solids);
  std::vector<int64_t> c_leaf(n_leaves * d), c_solid(n_solids * d);
  // independent per id; a failure is reported after the threads join
  std::atomic<bool> too_deep{false};
  auto decode_range = [&](const uint64_t* ids, std::vector<int>& lv, std::vector<int64_t>& cc) {
    return [&, ids](int64_t a, int64_t b) {
      for (int64_t i = a; i < b; ++i) {
        try {
          decode(ids[i], lv[i], &cc[i * d]);
        } catch (const MeshError&) {
          too_deep = true;
          return;
        }
      }
    };
  };
  parallel_for(n_leaves, decode_range(leaf_ids, lvl_leaf, c_leaf));
  parallel_for(n_solids, decode_range(solid_ids, lvl_solid, c_solid));
  if (too_deep) throw MeshError("treeID beyond the supported depth");
  int lmax = P.level0;
  for (int64_t i = 0; i < n_leaves; ++i) lmax = std::max(lmax, lvl_leaf[i]);
  for (int64_t i = 0; i < n_solids; ++i) lmax = std::max(lmax, lvl_solid[i]);
  const int L0 = P.level0, nlev = lmax - L0 + 1;
  std::vector<LevelWork> W(nlev);
  unsigned __int128 volume = 0;
  auto place = [&](int L, const int64_t* c, bool solid) {
    if (L < L0) throw MeshError("element coarser than level0");
    for (int a = 0; a < d; ++a)
      if (c[a] < g.lo(a, L) || c[a] >= g.hi(a, L))
        throw MeshError("element outside the domain box");
    auto& w = W[L - L0];
    auto& vec = solid ? w.solid : w.fluid;
    for (int a = 0; a < d; ++a) vec.push_back(c[a]);
    volume += (unsigned __int128)1 << (d * (lmax - L));
    // bounding boxes of this level and all coarser ones (ancestors)
    for (int K = L0; K <= L; ++K) {
      int64_t anc[3];
      for (int a = 0; a < d; ++a) anc[a] = c[a] >> (L - K);
      extend_bb(W[K - L0], anc, d);
      if (K < L) W[K - L0].deeper++;
    }
  };
  for (int64_t i = 0; i < n_leaves; ++i) place(lvl_leaf[i], &c_leaf[i * d], false);
  for (int64_t i = 0; i < n_solids; ++i) place(lvl_solid[i], &c_solid[i * d], true);
  unsigned __int128 box = 1;
  for (int a = 0; a < d; ++a) box *= (unsigned __int128)g.e[a];
  box <<= d * (lmax - L0);
  if (volume != box) throw MeshError("leaves and solids do not tile the domain box");

  T.mark("decode");
  // ---- level maps ---------------------------------------------------
  for (int k = 0; k < nlev; ++k) {
    const int L = L0 + k;
    auto& w = W[k];
    auto& m = w.map;
    m.d = d;
    m.L = L;
    unsigned __int128 vol = 1;
    for (int a = 0; a < d; ++a) {
      if (g.per[a] || !w.bb_set) {
        m.lo[a] = g.lo(a, L);
        m.ext[a] = g.hi(a, L) - g.lo(a, L);
      } else {
        const int64_t lo = std::max(g.lo(a, L), w.bb_lo[a] - 2);
        const int64_t hi = std::min(g.hi(a, L), w.bb_hi[a] + 3);
        m.lo[a] = lo;
        m.ext[a] = hi - lo;
      }
      vol *= (unsigned __int128)m.ext[a];
    }
    const int64_t count = (int64_t)(w.fluid.size() + w.solid.size()) / d + w.deeper;
    m.dense = vol <= (unsigned __int128)(16 * count + (1 << 24));
    if (m.dense) m.grid.assign((size_t)vol, V_EMPTY);
  }
  for (int k = 0; k < nlev; ++k) {
    auto& w = W[k];
    const int64_t nf = (int64_t)w.fluid.size() / d;
    for (int64_t i = 0; i < nf; ++i) {
      if (w.map.get(&w.fluid[i * d]) != V_EMPTY) throw MeshError("duplicate leaf");
      w.map.set(&w.fluid[i * d], (int32_t)i);
    }
    for (size_t i = 0; i < w.solid.size() / d; ++i) {
      if (w.map.get(&w.solid[i * d]) != V_EMPTY) throw MeshError("overlapping elements");
      w.map.set(&w.solid[i * d], V_SOLID);
    }
  }
  T.mark("insert");
  // refined positions: ancestors of every deeper leaf or solid
  auto mark_ancestors = [&](int L, const int64_t* c) {
    for (int K = L - 1; K >= L0; --K) {
      int64_t anc[3];
      for (int a = 0; a < d; ++a) anc[a] = c[a] >> (L - K);
      auto& m = W[K - L0].map;
      const int32_t v = m.get(anc);
      if (v == V_REFINED) return;  // coarser ancestors already marked
      if (v != V_EMPTY) throw MeshError("overlapping elements");
      m.set(anc, V_REFINED);
      for (int a = 0; a < d; ++a) W[K - L0].refined.push_back(anc[a]);
    }
  };
  for (int64_t i = 0; i < n_leaves; ++i) mark_ancestors(lvl_leaf[i], &c_leaf[i * d]);
  for (int64_t i = 0; i < n_solids; ++i) mark_ancestors(lvl_solid[i], &c_solid[i * d]);
  std::vector<int>().swap(lvl_leaf);
  std::vector<int64_t>().swap(c_leaf);

  T.mark("refined");
  // ---- ghost classification -------------------------------------------
  // GhostFromFiner(L): refined cells within L-infinity distance 1 of level-L
  // fluid.  The fluid cells within distance R = ceil(layers/2) of a refined
  // cell are the ring whose children are the only candidates for
  // GhostFromCoarser(L+1): a level-(L+1) position within distance `layers`
  // of level-(L+1) fluid has its parent within distance R of a refined
  // level-L cell.
  const int layers = P.gfc_layers, ring_r = (layers + 1) / 2;
  for (int k = 0; k < nlev; ++k) {
    const int L = L0 + k;
    auto& w = W[k];
    auto& m = w.map;
    const int64_t nf = (int64_t)w.fluid.size() / d;
    std::vector<char> ring_mark((size_t)nf, 0);
    const int64_t nr = (int64_t)w.refined.size() / d;
    for (int64_t r = 0; r < nr; ++r) {
      const int64_t* x = &w.refined[r * d];
      bool touches = false;
      for_offsets(d, ring_r, [&](const int64_t* o, int dist) {
        int64_t y[3];
        for (int a = 0; a < d; ++a) y[a] = x[a] + o[a];
        if (g.wrap(y, L)) return;
        const int32_t v = m.get(y);
        if (v >= 0) {
          if (dist == 1) touches = true;
          if (!ring_mark[v]) {
            ring_mark[v] = 1;
            for (int a = 0; a < d; ++a) w.ring.push_back(y[a]);
          }
        }
      });
      if (touches) {
        m.set(x, V_GFF);
        for (int a = 0; a < d; ++a) w.gff.push_back(x[a]);
      }
    }
  }
  for (int k = 1; k < nlev; ++k) {
    const int L = L0 + k;
    auto& w = W[k];
    auto& m = w.map;
    const auto& ring = W[k - 1].ring;
    const int nch = 1 << d;
    for (size_t r = 0; r < ring.size() / d; ++r) {
      for (int c = 0; c < nch; ++c) {
        int64_t y[3];
        for (int a = 0; a < d; ++a) y[a] = 2 * ring[r * d + a] + ((c >> a) & 1);
        if (m.get(y) != V_EMPTY) continue;
        int best = layers + 1;
        for_offsets(d, layers, [&](const int64_t* o, int dist) {
          if (dist >= best) return;
          int64_t z[3];
          for (int a = 0; a < d; ++a) z[a] = y[a] + o[a];
          if (g.wrap(z, L)) return;
          if (m.get(z) >= 0) best = dist;
        });
        if (best <= layers) {
          m.set(y, best < layers ? V_GFC_IN : V_GFC_OUT);
          for (int a = 0; a < d; ++a) w.gfc.push_back(y[a]);
        }
      }
    }
  }
  for (auto& w : W) {
    std::vector<int64_t>().swap(w.refined);
  }

  T.mark("classify");
  // ---- capture sources ----------------------------------------------
  // Fluid elements read by an interpolation (the parent H and K, M, N of a
  // GhostFromCoarser one level up, the four children of a GhostFromFiner one
  // level down) are laid out as the tail of the fluid segment, so the
  // stream-collide kernel knows from the index alone that it must record the
  // pre-collision moments of an element.
  std::vector<std::vector<char>> src_mark(nlev);
  for (int k = 0; k < nlev; ++k) src_mark[k].assign(W[k].fluid.size() / d, 0);
  for (int k = 1; k < nlev; ++k) {
    const auto& gl = W[k].gfc;
    for (size_t j = 0; j < gl.size() / d; ++j) {
      int64_t par[3], s[3];
      for (int a = 0; a < d; ++a) {
        par[a] = gl[j * d + a] >> 1;
        s[a] = (gl[j * d + a] & 1) ? 1 : -1;
      }
      int64_t off[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
      if (d == 3) {
        off[1][0] = s[0]; off[1][1] = s[1];
        off[2][0] = s[0]; off[2][2] = s[2];
        off[3][1] = s[1]; off[3][2] = s[2];
      } else {
        off[1][0] = s[0];
        off[2][1] = s[1];
        off[3][0] = s[0]; off[3][1] = s[1];
      }
      for (int t = 0; t < 4; ++t) {
        int64_t y[3];
        for (int a = 0; a < d; ++a) y[a] = par[a] + off[t][a];
        if (g.wrap(y, L0 + k - 1)) continue;  // rejected with the source check
        const int32_t v = W[k - 1].map.get(y);
        if (v >= 0) src_mark[k - 1][v] = 1;
      }
    }
  }
  for (int k = 0; k + 1 < nlev; ++k) {
    const auto& gl = W[k].gff;
    static const int ch3[4][3] = {{0, 0, 0}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}};
    static const int ch2[4][2] = {{0, 0}, {1, 0}, {0, 1}, {1, 1}};
    for (size_t j = 0; j < gl.size() / d; ++j)
      for (int t = 0; t < 4; ++t) {
        int64_t y[3];
        for (int a = 0; a < d; ++a) y[a] = 2 * gl[j * d + a] + (d == 3 ? ch3[t][a] : ch2[t][a]);
        const int32_t v = W[k + 1].map.get(y);
        if (v >= 0) src_mark[k + 1][v] = 1;
      }
  }

  // ---- layout -------------------------------------------------------
  P.lv.assign(nlev, LevelPlan());
  for (int k = 0; k < nlev; ++k) {
    const int L = L0 + k;
    auto& w = W[k];
    auto& lp = P.lv[k];
    lp.level = L;
    std::vector<int64_t> inner, outer, plain, capt;
    for (size_t i = 0; i < w.gfc.size() / d; ++i) {
      const int64_t* y = &w.gfc[i * d];
      auto& dst = (w.map.get(y) == V_GFC_IN) ? inner : outer;
      for (int a = 0; a < d; ++a) dst.push_back(y[a]);
    }
    for (size_t i = 0; i < w.fluid.size() / d; ++i) {
      auto& dst = src_mark[k][i] ? capt : plain;
      for (int a = 0; a < d; ++a) dst.push_back(w.fluid[i * d + a]);
    }
    std::vector<char>().swap(src_mark[k]);
    std::vector<int64_t> all;
    const std::vector<int64_t>* parts[5] = {&plain, &capt, &inner, &outer, &w.gff};
    int64_t counts[5];
    lp.tid.clear();
    for (int p = 0; p < 5; ++p) {
      const auto& v = *parts[p];
      const int64_t n = (int64_t)v.size() / d;
      counts[p] = n;
      std::vector<std::pair<uint64_t, int64_t>> key(n);
      parallel_for(n, [&](int64_t a, int64_t b) {
        for (int64_t i = a; i < b; ++i) key[i] = {morton(&v[i * d], d, L), i};
      });
      parallel_sort(key);
      const uint64_t first = level_first_id(L, d);
      const size_t t0 = lp.tid.size(), a0 = all.size();
      lp.tid.resize(t0 + n);
      all.resize(a0 + (size_t)n * d);
      parallel_for(n, [&](int64_t a, int64_t b) {
        for (int64_t i = a; i < b; ++i) {
          lp.tid[t0 + i] = first + key[i].first;
          for (int c = 0; c < d; ++c) all[a0 + (size_t)i * d + c] = v[key[i].second * d + c];
        }
      });
    }
    lp.cap_begin = counts[0];
    lp.n_fluid = counts[0] + counts[1];
    lp.n_inner = counts[2];
    lp.n_outer = counts[3];
    lp.n_gff = counts[4];
    lp.n = lp.n_fluid + lp.n_inner + lp.n_outer + lp.n_gff;
    if (lp.n >= INT32_MAX) throw MeshError("level has too many elements for int32 indices");
    lp.coords.resize((size_t)d * lp.n);
    for (int64_t i = 0; i < lp.n; ++i) {
      for (int a = 0; a < d; ++a) lp.coords[(size_t)a * lp.n + i] = (int32_t)all[i * d + a];
      w.map.set(&all[i * d], (int32_t)i);
    }
    std::vector<int64_t>().swap(w.gfc);
    std::vector<int64_t>().swap(w.gff);
    std::vector<int64_t>().swap(w.fluid);
    w.fluid.swap(all);  // keep layout-ordered coords
  }

  T.mark("layout");
  // ---- neighbours ----------------------------------------------------
  for (int k = 0; k < nlev; ++k) {
    const int L = L0 + k;
    auto& w = W[k];
    auto& lp = P.lv[k];
    const int64_t n = lp.n;
    lp.nbr.assign((size_t)(q - 1) * n, MLBM_NBR_MISSING);
    const CellMap& m = w.map;
    int64_t vel[27][3];
    int64_t delta[27];
    for (int i = 0; i < q; ++i) {
      int64_t v[3] = {0, 0, 0};
      for (int a = 0; a < d; ++a) v[a] = stencil_c(P.stencil, i, a);
      int64_t stride = 1;
      delta[i] = 0;
      for (int a = 0; a < d; ++a) {
        vel[i][a] = v[a];
        delta[i] += -v[a] * stride;
        stride *= m.ext[a];
      }
    }
    auto work = [&](int64_t x0, int64_t x1) {
      for (int64_t x = x0; x < x1; ++x) {
        const int64_t* cx = &w.fluid[x * d];
        bool interior = m.dense;
        for (int a = 0; a < d && interior; ++a)
          interior = cx[a] >= m.lo[a] + 1 && cx[a] < m.lo[a] + m.ext[a] - 1;
        if (interior) {
          const int64_t base = m.dkey(cx);
          for (int i = 1; i < q; ++i) {
            const int32_t val = m.grid[base + delta[i]];
            lp.nbr[(size_t)(i - 1) * n + x] =
                val >= 0 ? val : (val == V_SOLID ? MLBM_NBR_BOUNCE : MLBM_NBR_MISSING);
          }
          continue;
        }
        for (int i = 1; i < q; ++i) {
          int64_t y[3];
          for (int a = 0; a < d; ++a) y[a] = cx[a] - vel[i][a];
          const int crossed = g.wrap(y, L);
          int32_t code;
          if (crossed) {
            code = g.face_code(crossed);
          } else {
            const int32_t val = m.get(y);
            code = val >= 0 ? val : (val == V_SOLID ? MLBM_NBR_BOUNCE : MLBM_NBR_MISSING);
          }
          lp.nbr[(size_t)(i - 1) * n + x] = code;
        }
      }
    };
    parallel_for(n, work);
    const int64_t act = lp.n_active_max();
    for (int i = 1; i < q; ++i)
      for (int64_t x = 0; x < act; ++x)
        if (lp.nbr[(size_t)(i - 1) * n + x] == MLBM_NBR_MISSING) {
          char msg[160];
          snprintf(msg, sizeof msg, "level %d: updated element %llu lacks a neighbour", L,
                   (unsigned long long)lp.tid[x]);
          throw MeshError(msg);
        }
    for (int i = 1; i < q; ++i)
      for (int64_t x = 0; x < lp.n_fluid; ++x)
        if (lp.nbr[(size_t)(i - 1) * n + x] == MLBM_NBR_BOUNCE) {
          lp.bounce.push_back((int32_t)x);
          lp.bounce.push_back(i);
        }
    // reorder bounce pairs into [2][n] (element ascending within direction)
    std::vector<int32_t> b((size_t)lp.bounce.size());
    const int64_t nb = (int64_t)lp.bounce.size() / 2;
    for (int64_t j = 0; j < nb; ++j) {
      b[j] = lp.bounce[2 * j];
      b[nb + j] = lp.bounce[2 * j + 1];
    }
    lp.bounce.swap(b);
    compress_pull_table(lp, q, d, level_first_id(L, d));
  }

  T.mark("neighbours");
  // ---- interpolation sources -------------------------------------------
  static const int gff3[4][3] = {{0, 0, 0}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}};
  static const int gff2[4][2] = {{0, 0}, {1, 0}, {0, 1}, {1, 1}};
  for (int k = 0; k < nlev; ++k) {
    const int L = L0 + k;
    auto& lp = P.lv[k];
    const int64_t n = lp.n;
    // GhostFromFiner: four fluid children on L+1
    lp.gff_src.assign((size_t)4 * lp.n_gff, -1);
    for (int64_t j = 0; j < lp.n_gff; ++j) {
      const int64_t x = lp.n_fluid + lp.n_gfc() + j;
      for (int s = 0; s < 4; ++s) {
        int64_t ch[3];
        for (int a = 0; a < d; ++a)
          ch[a] = 2 * (int64_t)lp.coords[(size_t)a * n + x] + (d == 3 ? gff3[s][a] : gff2[s][a]);
        const int32_t v = W[k + 1].map.get(ch);
        if (v < 0 || v >= P.lv[k + 1].n_fluid)
          throw MeshError("GhostFromFiner source is not fluid");
        lp.gff_src[(size_t)s * lp.n_gff + j] = v;
      }
    }
    // GhostFromCoarser: parent H and K, M, N (3D) or the square (2D)
    const int64_t ng = lp.n_gfc();
    lp.gfc_src.assign((size_t)4 * ng, -1);
    if (ng) {
      const auto& cp = P.lv[k - 1];
      const int64_t cgff = cp.n_fluid + cp.n_gfc();
      for (int64_t j = 0; j < ng; ++j) {
        const int64_t x = lp.n_fluid + j;
        int64_t par[3], s[3];
        for (int a = 0; a < d; ++a) {
          const int64_t c = lp.coords[(size_t)a * n + x];
          par[a] = c >> 1;
          s[a] = (c & 1) ? 1 : -1;
        }
        int64_t off[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        if (d == 3) {
          off[1][0] = s[0]; off[1][1] = s[1];
          off[2][0] = s[0]; off[2][2] = s[2];
          off[3][1] = s[1]; off[3][2] = s[2];
        } else {
          off[1][0] = s[0];
          off[2][1] = s[1];
          off[3][0] = s[0]; off[3][1] = s[1];
        }
        for (int t = 0; t < 4; ++t) {
          int64_t y[3];
          for (int a = 0; a < d; ++a) y[a] = par[a] + off[t][a];
          if (g.wrap(y, L - 1)) throw MeshError("GhostFromCoarser source outside the domain");
          const int32_t v = W[k - 1].map.get(y);
          const bool fluid = v >= 0 && v < cp.n_fluid;
          const bool ghost_ff = v >= cgff;
          if (t == 0 ? !fluid : !(fluid || ghost_ff))
            throw MeshError("GhostFromCoarser source is not fluid or GhostFromFiner");
          lp.gfc_src[(size_t)t * ng + j] = v;
        }
      }
    }
  }

  T.mark("sources");
  // ---- capture sets, slots, parent groups -------------------------------
  std::vector<std::vector<int32_t>> slot_of(nlev);
  for (int k = 0; k < nlev; ++k) {
    auto& lp = P.lv[k];
    std::vector<char> mark((size_t)lp.n_fluid, 0);
    if (k + 1 < nlev) {
      const auto& fp = P.lv[k + 1];
      for (int32_t v : fp.gfc_src)
        if (v >= 0 && v < lp.n_fluid) mark[v] = 1;
    }
    if (k > 0) {
      const auto& cpl = P.lv[k - 1];
      for (int32_t v : cpl.gff_src)
        if (v >= 0 && v < lp.n_fluid) mark[v] = 1;
    }
    // the sources found in the tables are exactly the laid-out tail
    for (int64_t x = 0; x < lp.n_fluid; ++x)
      if ((bool)mark[x] != (x >= lp.cap_begin))
        throw MeshError("internal: capture segment does not match the source tables");
    slot_of[k].assign((size_t)lp.n, -1);
    lp.cap_elem.clear();
    for (int64_t x = lp.cap_begin; x < lp.n_fluid; ++x) {
      slot_of[k][x] = (int32_t)lp.cap_elem.size();
      lp.cap_elem.push_back((int32_t)x);
    }
    const int64_t gb = lp.n_fluid + lp.n_gfc();
    for (int64_t j = 0; j < lp.n_gff; ++j)
      slot_of[k][gb + j] = (int32_t)(lp.n_cap_fluid() + j);
  }
  for (int k = 0; k < nlev; ++k) {
    auto& lp = P.lv[k];
    lp.gff_slot.assign((size_t)4 * lp.n_gff, -1);
    for (size_t t = 0; t < lp.gff_src.size(); ++t) {
      lp.gff_slot[t] = slot_of[k + 1][lp.gff_src[t]];
      if (lp.gff_slot[t] < 0) throw MeshError("internal: GhostFromFiner source not captured");
    }
    const int64_t ng = lp.n_gfc();
    if (!ng) continue;
    const int L = L0 + k;
    const int64_t n = lp.n;
    // parents in ascending element order of the coarse level
    std::vector<std::pair<int32_t, int64_t>> par;  // (parent elem, ghost j)
    par.reserve(ng);
    for (int64_t j = 0; j < ng; ++j) par.emplace_back(lp.gfc_src[j], j);
    std::sort(par.begin(), par.end());
    const int NB = group_slots(d), NC = group_children(d);
    std::vector<int32_t> parents;
    for (size_t t = 0; t < par.size(); ++t)
      if (t == 0 || par[t].first != par[t - 1].first) parents.push_back(par[t].first);
    lp.n_groups = (int64_t)parents.size();
    lp.grp_src.assign((size_t)NB * lp.n_groups, -1);
    lp.grp_child.assign((size_t)NC * lp.n_groups, -1);
    const auto& cp = P.lv[k - 1];
    for (int64_t gi = 0; gi < lp.n_groups; ++gi) {
      const int32_t pe = parents[gi];
      int64_t pc[3];
      for (int a = 0; a < d; ++a) pc[a] = cp.coords[(size_t)a * cp.n + pe];
      for_offsets(d, 1, [&](const int64_t* o, int) {
        const int sl = group_slot_of(d, (int)o[0], (int)o[1], d == 3 ? (int)o[2] : 0);
        if (sl < 0) return;
        int64_t y[3];
        for (int a = 0; a < d; ++a) y[a] = pc[a] + o[a];
        if (g.wrap(y, L - 1)) return;
        const int32_t v = W[k - 1].map.get(y);
        if (v >= 0) lp.grp_src[(size_t)sl * lp.n_groups + gi] = slot_of[k - 1][v];
      });
      lp.grp_src[(size_t)group_parent_slot(d) * lp.n_groups + gi] = slot_of[k - 1][pe];
      // every source a present child uses must have a capture slot
      for (int c = 0; c < NC; ++c) {
        int64_t ch[3];
        for (int a = 0; a < d; ++a) ch[a] = 2 * pc[a] + ((c >> a) & 1);
        const int32_t v = W[k].map.get(ch);
        if (!(v >= lp.n_fluid && v < lp.n_fluid + ng)) continue;
        const int j = (int)(v - lp.n_fluid);
        for (int t = 0; t < 4; ++t) {
          const int32_t e = lp.gfc_src[(size_t)t * ng + j];
          int64_t o3[3] = {0, 0, 0};
          for (int a = 0; a < d; ++a) o3[a] = (int64_t)cp.coords[(size_t)a * cp.n + e] - pc[a];
          // undo the periodic wrap of the offset
          for (int a = 0; a < d; ++a) {
            const int64_t ext = g.hi(a, L - 1) - g.lo(a, L - 1);
            if (o3[a] > 1) o3[a] -= ext;
            if (o3[a] < -1) o3[a] += ext;
          }
          const int sl = group_slot_of(d, (int)o3[0], (int)o3[1], (int)o3[2]);
          if (sl < 0 || lp.grp_src[(size_t)sl * lp.n_groups + gi] != slot_of[k - 1][e] ||
              slot_of[k - 1][e] < 0)
            throw MeshError("internal: GhostFromCoarser source slot mismatch");
        }
      }
      for (int c = 0; c < NC; ++c) {
        int64_t ch[3];
        for (int a = 0; a < d; ++a) ch[a] = 2 * pc[a] + ((c >> a) & 1);
        const int32_t v = W[k].map.get(ch);
        if (v >= lp.n_fluid && v < lp.n_fluid + ng)
          lp.grp_child[(size_t)c * lp.n_groups + gi] = v;
      }
    }
    (void)n;
    (void)L;
    // staging rows of the synchronous fill (coarse GhostFromFiner records
    // are formed from their fine sources, whose slots the row carries)
    lp.grp_tab.assign((size_t)4 * NB * lp.n_groups, 0);
    const int64_t rec0 = cp.n_cap_fluid();
    for (int64_t e = 0; e < NB * lp.n_groups; ++e) {
      const int32_t s2 = lp.grp_src[e];
      int32_t* t = &lp.grp_tab[(size_t)4 * e];
      if (s2 >= rec0) {
        const int64_t j = s2 - rec0;
        for (int u = 0; u < 4; ++u) t[u] = cp.gff_slot[(size_t)u * cp.n_gff + j];
        t[0] = -2 - t[0];
      } else {
        t[0] = s2;
      }
    }
  }

  // ---- adjoint tables ------------------------------------------------------
  for (int k = 0; k < nlev; ++k) {
    auto& lp = P.lv[k];
    const int64_t n = lp.n, nf = lp.n_fluid;
    for (int v = 0; v < 2; ++v) {
      const int64_t act = v == 0 ? nf : nf + lp.n_inner;
      std::vector<char> hit((size_t)q * nf, 0);
      for (int64_t x = 0; x < act; ++x) {
        if (x < nf) hit[x] = 1;  // rest direction reads the element itself
        for (int i = 1; i < q; ++i) {
          const int32_t y = lp.nbr[(size_t)(i - 1) * n + x];
          if (y >= 0 && y < nf) hit[(size_t)i * nf + y] = 1;
          if (y == MLBM_NBR_BOUNCE && x < nf) {
            const int o = stencil_opp(P.stencil, i);
            hit[(size_t)o * nf + x] = 1;
          }
        }
      }
      auto& u = lp.unassigned[v];
      u.clear();
      std::vector<int32_t> dirs;
      for (int i = 0; i < q; ++i)
        for (int64_t x = 0; x < nf; ++x)
          if (!hit[(size_t)i * nf + x]) {
            u.push_back((int32_t)x);
            dirs.push_back(i);
          }
      u.insert(u.end(), dirs.begin(), dirs.end());
    }
    lp.copy_elems.clear();
    for (int64_t x = 0; x < lp.n_active_max(); ++x)
      for (int i = 1; i < q; ++i)
        if (lp.nbr[(size_t)(i - 1) * n + x] == MLBM_NBR_COPY) {
          lp.copy_elems.push_back((int32_t)x);
          break;
        }
    // GhostFromCoarser transpose: each parent group sums its children's
    // contributions per neighbourhood slot; coarse capture slot s then
    // gathers the rows (group * NB + slot) that refer to it
    lp.csr_ptr.clear();
    lp.csr_ent.clear();
    if (lp.n_gfc() && lp.n_groups) {
      const int NB = group_slots(d);
      const int64_t ncap_c = P.lv[k - 1].n_cap();
      std::vector<int32_t> count((size_t)ncap_c + 1, 0);
      for (int64_t g2 = 0; g2 < lp.n_groups; ++g2)
        for (int sl = 0; sl < NB; ++sl) {
          const int32_t s2 = lp.grp_src[(size_t)sl * lp.n_groups + g2];
          if (s2 >= 0) count[s2 + 1]++;
        }
      for (int64_t s2 = 0; s2 < ncap_c; ++s2) count[s2 + 1] += count[s2];
      lp.csr_ptr = count;
      lp.csr_ent.assign((size_t)count[ncap_c], 0);
      std::vector<int32_t> fillp(count.begin(), count.end() - 1);
      for (int64_t g2 = 0; g2 < lp.n_groups; ++g2)  // ascending (group, slot) in each row
        for (int sl = 0; sl < NB; ++sl) {
          const int32_t s2 = lp.grp_src[(size_t)sl * lp.n_groups + g2];
          if (s2 >= 0) lp.csr_ent[fillp[s2]++] = (int32_t)(g2 * NB + sl);
        }
    }
  }
  // a fine source belongs to exactly one GhostFromFiner (disjoint children)
  for (int k = 0; k + 1 < nlev; ++k) {
    std::vector<char> used((size_t)P.lv[k + 1].n_cap(), 0);
    for (int32_t sl : P.lv[k].gff_slot) {
      if (used[sl]) throw MeshError("internal: shared GhostFromFiner source");
      used[sl] = 1;
    }
  }
}

}  // namespace
}  // namespace mlbm

using namespace mlbm;

extern "C" {

const char* mlbm_error_string(int32_t code) {
  switch (code) {
    case MLBM_OK: return "ok";
    case MLBM_E_ARG: return "invalid argument";
    case MLBM_E_MESH: return "invalid mesh";
    case MLBM_E_STATE: return "call out of order";
    case MLBM_E_HIP: return "HIP runtime error";
    case MLBM_E_OOM: return "host out of memory";
    default: return "unknown error";
  }
}

const char* mlbm_last_error(void) { return g_last_error.c_str(); }

int32_t mlbm_lattice(int32_t stencil, int32_t* q, int32_t* c, double* w) {
  if (stencil != MLBM_D2Q9 && stencil != MLBM_D3Q19 && stencil != MLBM_D3Q27)
    return fail(MLBM_E_ARG, "unknown stencil %d", stencil);
  const int Q = stencil_q(stencil), D = stencil_d(stencil);
  if (q) *q = Q;
  for (int i = 0; i < Q; ++i) {
    for (int a = 0; a < D; ++a)
      if (c) c[i * D + a] = stencil_c(stencil, i, a);
    if (w) w[i] = stencil_w(stencil, i);
  }
  return MLBM_OK;
}

int32_t mlbm_set_morton_policy(double level_min_fraction, int32_t block_min_directions) {
  if (!(level_min_fraction >= 0.0 && level_min_fraction <= 1.0) || block_min_directions < 1 ||
      block_min_directions > 26)
    return fail(MLBM_E_ARG, "bad Morton policy (%g, %d)", level_min_fraction, block_min_directions);
  g_morton_level_min = level_min_fraction;
  g_morton_block_min = block_min_directions;
  return MLBM_OK;
}

int32_t mlbm_set_gfc_layers(int32_t layers) {
  if (layers != 2 && layers != 4) return fail(MLBM_E_ARG, "GhostFromCoarser layers must be 2 or 4");
  g_gfc_layers = layers;
  return MLBM_OK;
}

int32_t mlbm_plan_gfc_layers(const mlbm_plan* plan, int32_t* layers) {
  if (!plan || !layers) return fail(MLBM_E_ARG, "NULL argument");
  *layers = plan->gfc_layers;
  return MLBM_OK;
}

int32_t mlbm_plan_create(int32_t stencil, int32_t level0, const int32_t* box_origin,
                         const int32_t* box_extent, const int32_t* face_bc,
                         const uint64_t* leaf_ids, int64_t n_leaves,
                         const uint64_t* solid_ids, int64_t n_solids, mlbm_plan** out) {
  if (!out) return fail(MLBM_E_ARG, "out is NULL");
  *out = nullptr;
  if (stencil != MLBM_D2Q9 && stencil != MLBM_D3Q19 && stencil != MLBM_D3Q27)
    return fail(MLBM_E_ARG, "unknown stencil %d", stencil);
  if (!box_origin || !box_extent || !face_bc || (!leaf_ids && n_leaves) ||
      (!solid_ids && n_solids) || n_leaves <= 0 || n_solids < 0)
    return fail(MLBM_E_ARG, "bad mesh arrays");
  const int d = stencil_d(stencil);
  if (level0 < 0 || level0 > (d == 3 ? 20 : 30)) return fail(MLBM_E_ARG, "bad level0");
  for (int a = 0; a < d; ++a) {
    if (box_extent[a] <= 0 || box_origin[a] < 0 ||
        (int64_t)box_origin[a] + box_extent[a] > ((int64_t)1 << level0))
      return fail(MLBM_E_ARG, "domain box outside the root cube");
    if (face_bc[2 * a] < 0 || face_bc[2 * a] > 3 || face_bc[2 * a + 1] < 0 || face_bc[2 * a + 1] > 3)
      return fail(MLBM_E_ARG, "bad face kind");
    if ((face_bc[2 * a] == MLBM_FACE_PERIODIC) != (face_bc[2 * a + 1] == MLBM_FACE_PERIODIC))
      return fail(MLBM_E_ARG, "periodic faces must come in pairs");
  }
  std::unique_ptr<mlbm_plan> P;
  try {
    P.reset(new mlbm_plan());
    P->stencil = stencil;
    P->d = d;
    P->q = stencil_q(stencil);
    P->level0 = level0;
    for (int a = 0; a < d; ++a) {
      P->origin[a] = box_origin[a];
      P->extent[a] = box_extent[a];
    }
    for (int f = 0; f < 2 * d; ++f) P->faces[f] = face_bc[f];
    P->gfc_layers = g_gfc_layers;
    build_plan(*P, leaf_ids, n_leaves, solid_ids, n_solids);
  } catch (const MeshError& e) {
    return fail(MLBM_E_MESH, "%s", e.what());
  } catch (const std::bad_alloc&) {
    return fail(MLBM_E_OOM, "host allocation failed while building the plan");
  } catch (const std::exception& e) {
    return fail(MLBM_E_ARG, "%s", e.what());
  }
  *out = P.release();
  return MLBM_OK;
}

void mlbm_plan_destroy(mlbm_plan* plan) { delete plan; }

int32_t mlbm_plan_set_walls(mlbm_plan* plan, const uint64_t* ids, const int32_t* dirs,
                            const double* q, int64_t n) {
  if (!plan) return fail(MLBM_E_ARG, "plan is NULL");
  if (n < 0 || (n > 0 && (!ids || !dirs || !q))) return fail(MLBM_E_ARG, "bad wall arrays");
  const int Q = plan->q, d = plan->d, nl = plan->nlev();
  struct Link { int64_t x; int32_t j, x2; double q; };
  try {
    // fluid elements of each level by treeID (the fluid segment keeps the
    // interpolation sources at its end, so it is not sorted as a whole)
    std::vector<std::vector<std::pair<uint64_t, int64_t>>> by_id(nl);
    for (int k = 0; k < nl; ++k) {
      const LevelPlan& lp = plan->lv[k];
      by_id[k].resize((size_t)lp.n_fluid);
      for (int64_t x = 0; x < lp.n_fluid; ++x) by_id[k][x] = {lp.tid[x], x};
      std::sort(by_id[k].begin(), by_id[k].end());
    }
    std::vector<std::vector<Link>> per(nl);
    for (int64_t t = 0; t < n; ++t) {
      const int i = dirs[t];
      if (i < 1 || i >= Q) return fail(MLBM_E_ARG, "wall link %lld: direction %d", (long long)t, i);
      if (!(q[t] >= 0.0 && q[t] <= 1.0))
        return fail(MLBM_E_ARG, "wall link %lld: fraction %g outside [0, 1]", (long long)t, q[t]);
      int k = -1;
      for (int kk = 0; kk < nl; ++kk) {
        const int L = plan->lv[kk].level;
        if (ids[t] >= level_first_id(L, d) && ids[t] < level_first_id(L + 1, d)) k = kk;
      }
      const LevelPlan* lp = k >= 0 ? &plan->lv[k] : nullptr;
      int64_t x = -1;
      if (lp) {
        const auto& v = by_id[k];
        auto it = std::lower_bound(v.begin(), v.end(), std::make_pair(ids[t], (int64_t)-1));
        if (it != v.end() && it->first == ids[t]) x = it->second;
      }
      if (x < 0)
        return fail(MLBM_E_MESH, "wall link %lld: %llu is not a fluid leaf", (long long)t,
                    (unsigned long long)ids[t]);
      const int j = stencil_opp(plan->stencil, i);
      if (lp->nbr[(size_t)(j - 1) * lp->n + x] != MLBM_NBR_BOUNCE)
        return fail(MLBM_E_MESH, "wall link %lld: the neighbour of %llu along %d is not solid",
                    (long long)t, (unsigned long long)ids[t], i);
      const int32_t s2 = lp->nbr[(size_t)(i - 1) * lp->n + x];
      per[k].push_back({x, j, s2 >= 0 ? s2 : -1, q[t]});
    }
    std::vector<LevelPlan> next(nl);
    for (int k = 0; k < nl; ++k) {
      auto& v = per[k];
      std::sort(v.begin(), v.end(), [](const Link& a, const Link& b) {
        return a.x != b.x ? a.x < b.x : a.j < b.j;
      });
      for (size_t e = 1; e < v.size(); ++e)
        if (v[e].x == v[e - 1].x && v[e].j == v[e - 1].j)
          return fail(MLBM_E_ARG, "a wall link is given twice");
      LevelPlan& o = next[k];
      for (const Link& l : v) {
        o.wall.insert(o.wall.end(),
                      {(int32_t)l.x, l.j, l.x2, stencil_wclass(plan->stencil, l.j)});
        o.wall_q.push_back(l.q);
      }
      // device copy: an element's links (at most q - 1 < NBR_BLOCK) stay in
      // one chunk of NBR_BLOCK, the work-group that forms and writes them
      for (size_t e = 0; e < v.size();) {
        size_t f = e;
        while (f < v.size() && v[f].x == v[e].x) ++f;
        const size_t used = o.wall_dev_q.size() % NBR_BLOCK;
        if (used + (f - e) > (size_t)NBR_BLOCK)
          for (size_t p = used; p < (size_t)NBR_BLOCK; ++p) {
            o.wall_dev.insert(o.wall_dev.end(), {-1, 0, -1, 0});
            o.wall_dev_q.push_back(0.5);
          }
        for (; e < f; ++e) {
          o.wall_dev.insert(o.wall_dev.end(), o.wall.begin() + 4 * e, o.wall.begin() + 4 * e + 4);
          o.wall_dev_q.push_back(v[e].q);
        }
      }
      // transpose of the pre-pass: link t writes W = (o, x) = a W + b (o, x2)
      // + c (j, x) with (a, b, c) = (2q, 1 - 2q, 0) for q < 1/2 (x2 an
      // element; else (1, 0, 0)) and (1/(2q), 0, 1 - 1/(2q)) for q >= 1/2
      struct Term { int64_t key; int32_t sd, se; double coef, seed; bool own; };
      std::vector<Term> terms;
      const int64_t nn = plan->lv[k].n;
      for (const Link& l : v) {
        const int o = stencil_opp(plan->stencil, l.j);
        const double cox = stencil_c(plan->stencil, o, 0);
        double a = 1, b = 0, c = 0;
        if (l.q < 0.5) {
          if (l.x2 >= 0) { a = 2 * l.q; b = 1 - 2 * l.q; }
        } else {
          a = 1 / (2 * l.q);
          c = 1 - a;
        }
        const int64_t w = (int64_t)o * nn + l.x;
        terms.push_back({w, o, (int32_t)l.x, a, cox * (a - 1), true});
        if (b != 0) terms.push_back({(int64_t)o * nn + l.x2, o, (int32_t)l.x, b, cox * b, false});
        if (c != 0) terms.push_back({(int64_t)l.j * nn + l.x, o, (int32_t)l.x, c, cox * c, false});
      }
      std::stable_sort(terms.begin(), terms.end(),
                       [](const Term& p, const Term& q2) { return p.key < q2.key; });
      for (size_t e = 0; e < terms.size();) {
        size_t f = e;
        bool own = false;
        while (f < terms.size() && terms[f].key == terms[e].key) own |= terms[f++].own;
        o.wadj_ent.insert(o.wadj_ent.end(), {(int32_t)(terms[e].key / nn),
                                             (int32_t)(terms[e].key % nn), own ? 0 : 1, 0});
        o.wadj_ptr.push_back((int32_t)o.wadj_coef.size());
        for (; e < f; ++e) {
          o.wadj_src.insert(o.wadj_src.end(), {terms[e].sd, terms[e].se});
          o.wadj_coef.push_back(terms[e].coef);
          o.wadj_seed.push_back(terms[e].seed);
        }
      }
      if (!terms.empty()) o.wadj_ptr.push_back((int32_t)o.wadj_coef.size());
    }
    for (int k = 0; k < nl; ++k) {
      plan->lv[k].wall.swap(next[k].wall);
      plan->lv[k].wall_q.swap(next[k].wall_q);
      plan->lv[k].wall_dev.swap(next[k].wall_dev);
      plan->lv[k].wall_dev_q.swap(next[k].wall_dev_q);
      plan->lv[k].wadj_ent.swap(next[k].wadj_ent);
      plan->lv[k].wadj_ptr.swap(next[k].wadj_ptr);
      plan->lv[k].wadj_src.swap(next[k].wadj_src);
      plan->lv[k].wadj_coef.swap(next[k].wadj_coef);
      plan->lv[k].wadj_seed.swap(next[k].wadj_seed);
    }
  } catch (const std::bad_alloc&) {
    return fail(MLBM_E_OOM, "host allocation failed while setting walls");
  }
  return MLBM_OK;
}

int32_t mlbm_plan_levels(const mlbm_plan* plan, int32_t* n_levels, int32_t* level0) {
  if (!plan) return fail(MLBM_E_ARG, "plan is NULL");
  if (n_levels) *n_levels = plan->nlev();
  if (level0) *level0 = plan->level0;
  return MLBM_OK;
}

int32_t mlbm_plan_level_info(const mlbm_plan* plan, int32_t k, int64_t* out) {
  if (!plan || !out) return fail(MLBM_E_ARG, "NULL argument");
  if (k < 0 || k >= plan->nlev()) return fail(MLBM_E_ARG, "level index %d out of range", k);
  const auto& lp = plan->lv[k];
  out[MLBM_INFO_LEVEL] = lp.level;
  out[MLBM_INFO_N] = lp.n;
  out[MLBM_INFO_N_FLUID] = lp.n_fluid;
  out[MLBM_INFO_N_GFC_INNER] = lp.n_inner;
  out[MLBM_INFO_N_GFC_OUTER] = lp.n_outer;
  out[MLBM_INFO_N_GFF] = lp.n_gff;
  out[MLBM_INFO_N_CAP_FLUID] = lp.n_cap_fluid();
  out[MLBM_INFO_N_CAP] = lp.n_cap();
  out[MLBM_INFO_N_GFC_GROUPS] = lp.n_groups;
  out[MLBM_INFO_N_BOUNCE] = lp.n_bounce();
  out[MLBM_INFO_N_WALL] = lp.n_wall();
  return MLBM_OK;
}

int32_t mlbm_plan_export(const mlbm_plan* plan, int32_t k, int32_t table, void* host_dst,
                         size_t* bytes) {
  if (!plan || !bytes) return fail(MLBM_E_ARG, "NULL argument");
  if (k < 0 || k >= plan->nlev()) return fail(MLBM_E_ARG, "level index %d out of range", k);
  const auto& lp = plan->lv[k];
  const void* src = nullptr;
  size_t n = 0;
  switch (table) {
    case MLBM_TABLE_TREEID: src = lp.tid.data(); n = lp.tid.size() * 8; break;
    case MLBM_TABLE_COORDS: src = lp.coords.data(); n = lp.coords.size() * 4; break;
    case MLBM_TABLE_NBR: src = lp.nbr.data(); n = lp.nbr.size() * 4; break;
    case MLBM_TABLE_GFC_SRC: src = lp.gfc_src.data(); n = lp.gfc_src.size() * 4; break;
    case MLBM_TABLE_GFF_SRC: src = lp.gff_src.data(); n = lp.gff_src.size() * 4; break;
    case MLBM_TABLE_CAPTURE: src = lp.cap_elem.data(); n = lp.cap_elem.size() * 4; break;
    case MLBM_TABLE_BOUNCE: src = lp.bounce.data(); n = lp.bounce.size() * 4; break;
    case MLBM_TABLE_NBR16: src = lp.nbr16.data(); n = lp.nbr16.size() * 2; break;
    case MLBM_TABLE_NBASE: src = lp.nbase.data(); n = lp.nbase.size() * 4; break;
    case MLBM_TABLE_NBR_HDR: src = lp.nhdr.data(); n = lp.nhdr.size() * 4; break;
    case MLBM_TABLE_NBR_WIDE: src = lp.nbr_wide.data(); n = lp.nbr_wide.size() * 2; break;
    case MLBM_TABLE_WALL: src = lp.wall.data(); n = lp.wall.size() * 4; break;
    case MLBM_TABLE_WALL_Q: src = lp.wall_q.data(); n = lp.wall_q.size() * 8; break;
    default: return fail(MLBM_E_ARG, "unknown table %d", table);
  }
  if (!host_dst) {
    *bytes = n;
    return MLBM_OK;
  }
  if (*bytes != n) return fail(MLBM_E_ARG, "table size is %zu bytes, got %zu", n, *bytes);
  if (n) memcpy(host_dst, src, n);
  return MLBM_OK;
}

}  // extern "C"
