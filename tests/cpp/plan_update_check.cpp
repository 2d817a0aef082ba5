// Re-planning in place (update_next_level) against planning afresh
// (plan_next_level): for structured grids in 2D and 3D, plan every level with
// one set of ranks, then walk the levels again with other ranks, updating
// each next level in place, and compare every descriptor table, size, slot
// list and copy map with a plan made afresh with the second ranks.  Exit
// status 0 when all match.
#include "sgf_plan.hpp"

#include <cstdio>
#include <cstdlib>
#include <cstring>

using namespace sgf;

template <typename V>
static bool same(const std::vector<V>& a, const std::vector<V>& b) {
  return a.size() == b.size() && (a.empty() || std::memcmp(a.data(), b.data(), a.size() * sizeof(V)) == 0);
}

static void grid_csr(int dim, const int* g, int dpn, std::vector<int64_t>& rp, std::vector<int32_t>& ci) {
  const int64_t nn = (int64_t)g[0] * g[1] * (dim == 3 ? g[2] : 1), n = nn * dpn;
  rp.assign(n + 1, 0);
  ci.clear();
  for (int64_t v = 0; v < nn; ++v) {
    const int x = v % g[0], y = (v / g[0]) % g[1], z = dim == 3 ? (int)(v / ((int64_t)g[0] * g[1])) : 0;
    for (int c = 0; c < dpn; ++c) {
      for (int dz = (dim == 3 ? -1 : 0); dz <= (dim == 3 ? 1 : 0); ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            const int X = x + dx, Y = y + dy, Z = z + dz;
            if (X < 0 || Y < 0 || Z < 0 || X >= g[0] || Y >= g[1] || (dim == 3 && Z >= g[2])) continue;
            if (dpn == 1 && std::abs(dx) + std::abs(dy) + std::abs(dz) > 1) continue;
            const int64_t u = X + (int64_t)g[0] * (Y + (int64_t)g[1] * Z);
            for (int c2 = 0; c2 < dpn; ++c2) ci.push_back((int32_t)(u * dpn + c2));
          }
      rp[v * dpn + c + 1] = (int64_t)ci.size();
    }
  }
}

// ranks of a level's compressions: a deterministic pattern per variant
static void set_ranks(Level& L, int variant) {
  L.rank.assign(L.comp.size(), 0);
  for (size_t c = 0; c < L.comp.size(); ++c) {
    const int full = std::min(L.comp[c].s, L.comp[c].c);
    const int drop = variant == 0 ? (int)(c % 3) : (int)((c * 7 + L.t) % 5);
    L.rank[c] = std::max(1, full - drop);
  }
}

// The destinations the device coarsening computes (coarsen_dest from the
// structure tables, each separator's father and first row, the ranks) equal
// the host copy lists, entry for entry, and lie inside the new level's arena
// and Phi.
static bool device_dest_match(const Level& C, const Level& N, const std::vector<CopyDesc>& bm,
                              const std::vector<CopyDesc>& pm, int pi) {
  std::vector<CoarsenPair> cp;
  std::vector<CoarsenSep> cs;
  coarsen_tables(C, N, cp, cs);
  if (N.cp_father.size() != C.seps.size() || N.cp_loc.size() != C.seps.size()) return false;
  const int64_t n_elems = N.front_elems + N.blk_elems;
  size_t at = 0;
  for (size_t q = 0; q < C.pairs.size(); ++q) {
    const PairDesc& pd = C.pairs[q];
    const int ra = C.post_size(pd.a), rb = C.post_size(pd.b);
    if (ra == 0 || rb == 0) continue;
    const CoarsenDst d = coarsen_dest(cp[q].kind, cp[q].tgt, cp[q].e, N.cp_loc[cp[q].pa], N.cp_loc[cp[q].pb],
                                      pd.a == pd.b, N.elim.data(), N.pairs.data(), N.nbr_off.data(), N.front_elems);
    for (int mode = 0; mode < 2; ++mode) {
      const int64_t dst = mode == 0 ? d.d0 : d.d1;
      if (dst < 0) continue;
      if (at >= bm.size()) return false;
      const CopyDesc& c = bm[at++];
      if (c.mode != mode || c.dst_off != dst || c.dst_ld != d.ld || c.rows != ra || c.cols != rb ||
          c.src_off != C.front_elems + pd.blk_off)
        return false;
      const int64_t last = mode == 0 ? dst + (ra - 1) + (int64_t)(rb - 1) * d.ld : dst + (rb - 1) + (int64_t)(ra - 1) * d.ld;
      if (dst < 0 || last >= n_elems) return false;
    }
  }
  if (at != bm.size()) return false;
  if (N.top) return pm.empty();
  size_t ap = 0;
  for (size_t p = 0; p < C.seps.size(); ++p) {
    const int a = cs[p].cluster;
    const int r = C.post_size(a);
    if (r == 0) continue;
    if (ap >= pm.size()) return false;
    const CopyDesc& c = pm[ap++];
    const int D = N.cp_father[p];
    if (c.src_off != C.phi_off[a] || c.src_ld != C.size[a] || c.rows != r || c.cols != pi ||
        c.dst_off != N.phi_off[D] + N.cp_loc[p] || c.dst_ld != N.size[D])
      return false;
  }
  return ap == pm.size();
}

static bool same_level(const Level& a, const Level& b) {
  return a.top == b.top && same(a.cell, b.cell) && same(a.size, b.size) && same(a.slot_ptr, b.slot_ptr) &&
         same(a.slots, b.slots) && same(a.nbr_off, b.nbr_off) && same(a.elim, b.elim) && same(a.nslots, b.nslots) &&
         same(a.pairs, b.pairs) && same(a.schur, b.schur) && same(a.comp, b.comp) && same(a.comp_nbr, b.comp_nbr) &&
         same(a.phi_off, b.phi_off) && same(a.sepacc, b.sepacc) && same(a.sepacc_src, b.sepacc_src) &&
         a.front_elems == b.front_elems && a.blk_elems == b.blk_elems && a.scratch_elems == b.scratch_elems &&
         a.t_elems == b.t_elems && a.cf_elems == b.cf_elems && a.n_elems == b.n_elems &&
         a.ltphi_elems == b.ltphi_elems && a.tau_elems == b.tau_elems && a.tb_elems == b.tb_elems &&
         a.phi_elems == b.phi_elems && a.max_front_rows == b.max_front_rows && a.max_cf_rows == b.max_cf_rows &&
         a.max_c == b.max_c && a.max_s == b.max_s && a.n_active == b.n_active && same(a.cp_father, b.cp_father) &&
         same(a.cp_loc, b.cp_loc);
}

int main() {
  // scheme: 0 Nest-All-All, 2 Nest-2-2 (N columns depend on the neighbours'
  // sizes), 3 Gen-All-All; compression 1: the low-rank equivalent
  struct Case {
    int dim, g[3], dpn, q, leaf, scheme, compression;
  } cases[] = {{2, {64, 64, 1}, 1, 1, 8, 0, 0},   {2, {200, 173, 1}, 1, 2, 8, 0, 0}, {3, {24, 22, 21}, 1, 1, 4, 0, 0},
               {3, {13, 12, 12}, 3, 1, 3, 0, 0}, {2, {61, 58, 1}, 1, 2, 4, 0, 0},  {2, {9, 7, 1}, 1, 0, 2, 0, 0},
               {2, {61, 58, 1}, 1, 2, 4, 2, 0},  {3, {24, 22, 21}, 1, 1, 4, 2, 0}, {2, {61, 58, 1}, 1, 1, 4, 3, 0},
               {3, {13, 12, 12}, 3, 1, 3, 3, 0}, {2, {61, 58, 1}, 1, 2, 4, 0, 1}, {3, {24, 22, 21}, 1, 1, 4, 2, 1},
               {2, {512, 512, 1}, 1, 2, 16, 0, 0}};
  int bad = 0;
  for (const Case& cs : cases) {
    Plan base;
    base.opt.dim = cs.dim;
    for (int a = 0; a < 3; ++a) base.opt.grid[a] = cs.g[a];
    base.opt.dpn = cs.dpn;
    base.opt.q = cs.q;
    base.opt.leaf = cs.leaf;
    base.opt.scheme = cs.scheme;
    base.opt.compression = cs.compression;
    base.n_nodes = (int64_t)cs.g[0] * cs.g[1] * (cs.dim == 3 ? cs.g[2] : 1);
    base.n = base.n_nodes * cs.dpn;
    base.pi = poly_cols(cs.dim, cs.q, cs.dpn);
    std::vector<int64_t> rp;
    std::vector<int32_t> ci;
    grid_csr(cs.dim, cs.g, cs.dpn, rp, ci);
    plan_level1(base, rp.data(), ci.data());
    // afresh with ranks of each variant
    Plan fresh[2] = {base, base};
    std::vector<std::vector<CopyDesc>> maps[2][2];
    for (int v = 0; v < 2; ++v) {
      std::vector<CopyDesc> bm, pm;
      while (!fresh[v].levels.back().top) {
        set_ranks(fresh[v].levels.back(), v);
        plan_next_level(fresh[v], bm, pm);
        maps[v][0].push_back(bm);
        maps[v][1].push_back(pm);
        const size_t li = fresh[v].levels.size() - 2;
        if (!device_dest_match(fresh[v].levels[li], fresh[v].levels[li + 1], bm, pm, base.pi)) {
          std::printf("case %dx%dx%d: device coarsening destinations differ at level %zu\n", cs.g[0], cs.g[1],
                      cs.g[2], li + 2);
          ++bad;
        }
      }
    }
    // in place: variant 0 afresh, then 1, then 0 again, level by level
    Plan P = base;
    {
      std::vector<CopyDesc> bm, pm;
      while (!P.levels.back().top) {
        set_ranks(P.levels.back(), 0);
        plan_next_level(P, bm, pm);
      }
    }
    int levels = 0, updated = 0;
    for (int v : {1, 0}) {
      bool ok = P.levels.size() == fresh[v].levels.size();
      for (size_t li = 0; ok && li + 1 < P.levels.size(); ++li) {
        set_ranks(P.levels[li], v);
        std::vector<CopyDesc> bm, pm;
        if (!update_next_level(P, li, bm, pm)) {
          std::printf("case %dx%dx%d: update refused at level %zu\n", cs.g[0], cs.g[1], cs.g[2], li + 1);
          ok = false;
          break;
        }
        ++updated;
        ok = same_level(P.levels[li + 1], fresh[v].levels[li + 1]) && same(bm, maps[v][0][li]) &&
             same(pm, maps[v][1][li]) && device_dest_match(P.levels[li], P.levels[li + 1], bm, pm, base.pi);
        if (!ok) std::printf("case %dx%dx%d: variant %d differs at level %zu\n", cs.g[0], cs.g[1], cs.g[2], v, li + 2);
      }
      levels = (int)P.levels.size();
      bad += ok ? 0 : 1;
    }
    std::printf("case %dx%dx%d dpn %d q %d leaf %d scheme %d compression %d: %d levels, %d in-place updates\n",
                cs.g[0], cs.g[1], cs.g[2], cs.dpn, cs.q, cs.leaf, cs.scheme, cs.compression, levels, updated);
  }
  std::printf(bad ? "MISMATCH\n" : "ok\n");
  return bad ? 1 : 0;
}
