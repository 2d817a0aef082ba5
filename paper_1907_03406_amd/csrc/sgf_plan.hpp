// Host-side symbolic planner of the SGF factorization (integer work only).
//
// Builds, level by level, the nodes (B, active set) of the nested-dissection
// partition hierarchy (Sec. 5.1, Defs. 2.1-2.4), the interior / separator
// split, the fill pattern created by eliminating the interiors (Eq. 4.2),
// the neighbour lists used by the compressions (Eq. 4.5) and the maps that
// carry the coarse blocks of one level into the nodes of the next (Sec. 4.3,
// Eq. 4.7).  Every array here is plain integers; the device kernels get them
// as descriptor tables.
#pragma once

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

// Functions shared by the planner (host) and the copy kernels (device).
#if defined(__HIPCC__)
#define SGF_HD __host__ __device__
#else
#define SGF_HD
#endif

namespace sgf {

struct Options {
  int dim = 2;
  int grid[3] = {1, 1, 1};
  int dpn = 1;
  int q = 1;
  int leaf = 8;
  int scheme = 0;
  int compress = 1;
  int compress_from_level = 1;
  int stop_rule = 0;
  int precision = 0;
  double rank_tol = 1e-12;
  // 0: polynomial compression (Eq. 3.2); 1: the standard low-rank
  // equivalent (Sec. 7.4, Eq. 7.5): Q from the pivoted QR of the scaled
  // off-diagonal block itself, cut at ranks recorded beforehand
  int compression = 0;
};

// Schemes (Sec. 5): which separator cells are compressed and how.
enum { SCHEME_NEST_ALL_ALL = 0, SCHEME_NEST_2_ALL = 1, SCHEME_NEST_2_2 = 2, SCHEME_GEN_ALL_ALL = 3 };

inline int poly_cols(int dim, int q, int dpn) {
  int p0 = q == 0 ? 1 : (q == 1 ? 1 + dim : (dim == 2 ? 6 : 10));
  return p0 * dpn;
}

// Per-axis classes at period d (Sec. 5.1): index i is on a cutting slab iff
// (i + 1) % d == 0 and i <= N - 2; class = 2 * (#slabs below) + [on slab].
struct Axis {
  std::vector<int32_t> cls;
  int32_t K = 1;
  std::vector<int32_t> rep;  // first index of each class
};

// General partition (Sec. 5.2): boxes of d consecutive vertices per axis
// (the last one shorter when d does not divide N); class = i / d.
inline Axis axis_boxes(int N, int d) {
  Axis a;
  a.cls.resize(N);
  for (int i = 0; i < N; ++i) a.cls[i] = i / d;
  a.K = (N + d - 1) / d;
  a.rep.assign(a.K, -1);
  for (int i = N - 1; i >= 0; --i) a.rep[a.cls[i]] = i;
  return a;
}

inline Axis axis_classes(int N, int d) {
  Axis a;
  a.cls.resize(N);
  int below = 0;
  for (int i = 0; i < N; ++i) {
    bool slab = ((i + 1) % d == 0) && (i <= N - 2);
    a.cls[i] = 2 * below + (slab ? 1 : 0);
    if (slab) ++below;
  }
  a.K = 2 * below + 1;
  a.rep.assign(a.K, -1);
  for (int i = N - 1; i >= 0; --i) a.rep[a.cls[i]] = i;
  return a;
}

struct Partition {
  int d = 0;
  int dim = 2;
  bool general = false;   // boxes of a general partition: every cell is compressed, none is an interior
  Axis ax[3];
  int64_t ncells = 1;
  bool is_root = false;
  int64_t cell_of(int ix, int iy, int iz) const {
    int64_t c = ax[0].cls[ix];
    if (dim >= 2) c += (int64_t)ax[0].K * ax[1].cls[iy];
    if (dim >= 3) c += (int64_t)ax[0].K * ax[1].K * ax[2].cls[iz];
    return c;
  }
  void split(int64_t cid, int cls[3]) const {
    cls[0] = (int)(cid % ax[0].K);
    cid /= ax[0].K;
    cls[1] = dim >= 2 ? (int)(cid % ax[1].K) : 0;
    cid /= (dim >= 2 ? ax[1].K : 1);
    cls[2] = dim >= 3 ? (int)cid : 0;
  }
  int type_of(int64_t cid) const {
    if (general) return 1;
    int c[3];
    split(cid, c);
    int t = 0;
    for (int a = 0; a < dim; ++a) t += c[a] & 1;
    return t;
  }
};

inline Partition make_partition(const Options& o, int d) {
  Partition p;
  p.d = d;
  p.dim = o.dim;
  p.general = o.scheme == SCHEME_GEN_ALL_ALL;
  p.ncells = 1;
  bool root = true;
  for (int a = 0; a < o.dim; ++a) {
    p.ax[a] = p.general ? axis_boxes(o.grid[a], d) : axis_classes(o.grid[a], d);
    p.ncells *= p.ax[a].K;
    if (p.ax[a].K > 1) root = false;
  }
  p.is_root = root;
  return p;
}

// Whether cell Y lies on the boundary of cell B in a nested-dissection
// partition (Sec. 5.1): Y != B, Y has B's class on every axis where B is a
// slab (odd class) and a class within one of B's on every other axis -- the
// edges and corners around a face, the two end corners of a 2D edge.
inline bool on_boundary(const Partition& p, int64_t B, int64_t Y) {
  if (B == Y || p.general) return false;
  int cb[3], cy[3];
  p.split(B, cb);
  p.split(Y, cy);
  for (int a = 0; a < p.dim; ++a) {
    if ((cb[a] & 1) && cy[a] != cb[a]) return false;
    if (std::abs(cy[a] - cb[a]) > 1) return false;
  }
  return true;
}

// Father of a cell of partition `lo` in the coarser partition `hi` (Sec. 4.3).
inline int64_t father_cell(const Partition& lo, const Partition& hi, int64_t cid) {
  int c[3];
  lo.split(cid, c);
  int idx[3] = {0, 0, 0};
  for (int a = 0; a < lo.dim; ++a) idx[a] = lo.ax[a].rep[c[a]];
  return hi.cell_of(idx[0], idx[1], idx[2]);
}

// Coarsening computed on the device (Secs. 4.3-4.4): for every pair block of
// the level below, where it goes in the new level (the kinds of
// emit_copy_maps: 0 diagonal block of an interior front, 1 diagonal pair
// block, 2 / 3 an interior front's neighbour rows (a's / b's father is the
// interior), 4 / 5 an off-diagonal pair block, a's father first / second),
// the target (front or pair index), the adjacency entry of the neighbour
// rows, and the separator positions of a and b; for every separator of the
// level below, its cluster and compression index.  These depend only on the
// structure, not on the ranks.
struct CoarsenPair {
  int64_t e;
  int32_t kind, tgt, pa, pb;
};
struct CoarsenSep {
  int32_t cluster, ci;
};

// Block copy: dst[(dr + i) + (dc + j) * dld] = src[i + j * sld] (mode 0) or
// dst[(dr + j) + (dc + i) * dld] (mode 1, transposed), i < rows, j < cols.
struct CopyDesc {
  int64_t src_off;   // absolute offset in the source buffer
  int64_t dst_off;   // absolute offset in the destination buffer, (dr, dc) included
  int32_t src_ld, dst_ld, rows, cols, mode, pad;
};

// Interior elimination (Eq. 4.2) on a front of (m + k) x (m + k), column
// major, whose first m columns become [L_I ; W^T] and whose trailing k x k
// lower triangle receives -W^T W.
struct ElimDesc {
  int64_t front_off;
  int64_t slot_off;     // slots of I (m entries)
  int64_t nslot_off;    // slots of the neighbours, concatenated (k entries)
  int64_t t_off;        // apply scratch (k entries per right-hand side)
  int32_t m, k, cluster;
  int32_t bw;           // lower bandwidth of M_II in slot order (m: dense); the
                        // Cholesky factor keeps it, so L_I is zero below it
  int64_t pk_off;       // packed copy of the factor for the apply sweeps (-1: none)
};

// One Schur contribution: dst pair block (ld = s_a) += front lower part.
struct SchurDesc {
  int64_t src_off;      // front_off + (m + off_b) + (m + off_a) * ld  [a < b]
  int32_t src_ld, diag;
};
struct PairDesc {
  int64_t blk_off;
  int64_t scratch_off;
  int32_t a, b;         // separator cluster indices (a <= b)
  int32_t s_a, s_b;
  int32_t ca, cb;       // compression indices or -1
  int32_t row_in_a, row_in_b;  // row of b inside a's compression front, and vice versa
  int32_t c_ptr, c_cnt; // Schur contributions
};

// Destination in the new level's arena of a pair block of the level below
// (CoarsenPair kinds, as in emit_copy_maps): d0 receives the block (element
// (i, j) at d0 + i + j ld), d1 its transpose (element (i, j) at d1 + j + i ld),
// -1 when not used.  oa / ob: first rows of a / b in their fathers; diag: the
// block is a diagonal pair block (a == b); NE / NP / nbr_off: the new level's
// interior fronts, pair blocks and neighbour offsets; n_front: the size of
// the fronts part of its arena (pair blocks follow).
struct CoarsenDst {
  int64_t d0, d1, ld;
};
SGF_HD inline CoarsenDst coarsen_dest(int kind, int tgt, int64_t e, int oa, int ob, bool diag,
                                      const ElimDesc* NE, const PairDesc* NP, const int32_t* nbr_off,
                                      int64_t n_front) {
  CoarsenDst r{-1, -1, 1};
  if (kind == 0 || kind == 1) {
    int64_t base;
    if (kind == 0) {
      base = NE[tgt].front_off;
      r.ld = (int64_t)NE[tgt].m + NE[tgt].k;
    } else {
      base = n_front + NP[tgt].blk_off;
      r.ld = NP[tgt].s_a;
    }
    r.d0 = base + oa + (int64_t)ob * r.ld;
    if (!diag) r.d1 = base + ob + (int64_t)oa * r.ld;
  } else if (kind == 2 || kind == 3) {
    r.ld = (int64_t)NE[tgt].m + NE[tgt].k;
    const int64_t row = NE[tgt].m + nbr_off[e];
    if (kind == 2) r.d1 = NE[tgt].front_off + (row + ob) + (int64_t)oa * r.ld;
    else r.d0 = NE[tgt].front_off + (row + oa) + (int64_t)ob * r.ld;
  } else if (kind == 4 || kind == 5) {
    r.ld = NP[tgt].s_a;
    if (kind == 4) r.d0 = n_front + NP[tgt].blk_off + oa + (int64_t)ob * r.ld;
    else r.d1 = n_front + NP[tgt].blk_off + ob + (int64_t)oa * r.ld;
  }
  return r;
}

// Compression of one separator B (Eqs. 3.1-3.5).
struct CompDesc {
  int64_t cf_off;       // compression front (s + K) x s, column major
  int64_t n_off;        // N buffer s x c (holds the reflectors afterwards)
  int64_t phi_off;      // Phi_B, s x pi (ld s); receives Q1^T L^T Phi_B
  int64_t ltphi_off;    // scratch s x pi
  int64_t tau_off;      // c entries
  int64_t slot_off;     // slots of B
  int32_t s, K, c, nnb, nb_ptr, cluster;
  int32_t self_cols;    // columns of L_B^T Phi_B at the start of N (pi; 0 for the low-rank equivalent)
  int64_t blk_diag;     // offset of M_BB pair block
  int64_t tb_off;       // s x s slot for T_B = Q^T L_B^{-1} (filled when the separator compresses)
};
// Columns of N that neighbour X contributes (Eq. 4.5): Mhat_BX Phi_X (pi
// columns), or Mhat_BX itself (s_X columns, `full`) for a cell on B's
// boundary in Nest-2-2 (Sec. 5.1) and for every neighbour in the low-rank
// equivalent (Eq. 7.5).
struct CompNbr {
  int64_t blk_off;      // pair block holding M_BX (if X > B) or M_XB (X < B)
  int64_t phi_off;      // Phi_X (ld s_X)
  int32_t s_x, trans, row, full;  // trans = 1: block stored as M_BX (s x s_X)
  int32_t col, pad;     // first column in N
};

// Apply of one compressed separator: y_B <- Q^T L_B^{-1} y_B and back.
struct CompApply {
  int64_t cf_off;
  int64_t v_off;
  int64_t tau_off;
  int64_t slot_off;
  int64_t t_off;        // explicit T_B = Q^T L_B^{-1} (s x s, column major)
  int32_t s, ld, r;
  int32_t v_off2;       // offset in the level's apply vector of compressed unknowns (s entries)
};

// Apply: separator S collects -sum_I (W_I^T y_I)[S part] from the interiors.
struct SepAcc {
  int64_t slot_off;
  int32_t s, c_ptr, c_cnt, pad;
};

struct Level {
  int t = 1;                  // 1-based level
  bool top = false;
  bool compress = false;
  // active clusters, ascending cell id
  std::vector<int64_t> cell;
  std::vector<int32_t> type, size;
  std::vector<int64_t> slot_ptr;
  std::vector<int32_t> slots;
  // pre-elimination adjacency (CSR, ascending); for an interior its entries
  // are its neighbours and nbr_off gives each one's offset in the front's k part
  std::vector<int64_t> adj_ptr;
  std::vector<int32_t> adj_idx;
  std::vector<int32_t> nbr_off;
  // interiors
  std::vector<int32_t> interiors;
  std::vector<int32_t> elim_of;            // cluster -> interior index or -1
  std::vector<ElimDesc> elim;
  std::vector<int32_t> nslots;             // neighbour slots of every interior
  int64_t front_elems = 0;
  int64_t t_elems = 0;                     // apply scratch per rhs
  int32_t max_front_rows = 0;
  // separators
  std::vector<int32_t> seps;
  std::vector<int32_t> sep_pos;            // cluster -> position in seps or -1
  // post-elimination separator adjacency (CSR by separator position,
  // ascending cluster ids); sadj_pair = pair id of (a, b) when b > a
  std::vector<int64_t> sadj_ptr;
  std::vector<int32_t> sadj_idx, sadj_pair, pair_diag;
  std::vector<PairDesc> pairs;
  std::vector<SchurDesc> schur;
  int64_t blk_elems = 0;
  int64_t scratch_elems = 0;
  // compression
  std::vector<int32_t> comp_of;            // cluster -> compression index or -1
  std::vector<CompDesc> comp;
  std::vector<CompNbr> comp_nbr;
  int64_t cf_elems = 0, n_elems = 0, ltphi_elems = 0, tau_elems = 0, tb_elems = 0;
  int32_t max_cf_rows = 0, max_c = 0, max_s = 0;
  // Phi per cluster
  std::vector<int64_t> phi_off;
  int64_t phi_elems = 0;
  // apply
  std::vector<SepAcc> sepacc;
  std::vector<int64_t> sepacc_src;         // t_off + offset of S in the interior's k part
  // results of the numeric phase
  std::vector<int32_t> rank;               // per compression
  std::vector<int32_t> planned_rank;       // ranks the next level was planned with
  std::vector<int32_t> active_pairs;       // pairs touching a compressed separator
  std::vector<int64_t> t_of_comp;          // offset of T_B per compression (-1: not compressed)
  std::vector<CompApply> capply;
  std::vector<int32_t> cap_of_acc;         // per SepAcc: its index in capply, or -1 (not compressed)
  bool acc_covers_capply = false;          // every compressed separator has a SepAcc
  int64_t n_active = 0;
  // structure recorded by build_level, from which build_offsets re-derives
  // every size-dependent field when only the cluster sizes change
  std::vector<int32_t> schur_ii;             // per Schur entry: interior index
  std::vector<int64_t> schur_ex, schur_ey;   //   and its adjacency entries x <= y
  std::vector<int32_t> cnbr_x, cnbr_pid;     // per compression neighbour: cluster, pair id
  std::vector<uint8_t> cnbr_full;            //   and whether it enters N whole
  std::vector<int32_t> pair_rowa, pair_rowb; // per pair: neighbour entry giving row_in_a / row_in_b (-1: none)
  std::vector<int32_t> sacc_p;               // per SepAcc: separator position
  std::vector<int32_t> sacc_ii;              // per sepacc_src entry: interior index
  std::vector<int64_t> sacc_e;               //   and adjacency entry
  // levels above the first: where the separators of the level below go
  // (father before a top merge) and where each pair block of the level below
  // is copied (kind, interior index or pair id, adjacency entry of the row)
  std::vector<int32_t> from_father;
  int32_t from_nfathers = 0;
  bool from_merged = false;
  std::vector<int8_t> cp_kind;
  std::vector<int32_t> cp_tgt;
  std::vector<int64_t> cp_e;
  bool can_update = false;
  // the father (index in this level) and first row there of every separator
  // of the level below, for the current sizes (the device coarsening
  // computes each block's destination from these, CoarsenPair, CoarsenSep)
  std::vector<int32_t> cp_father, cp_loc;

  int32_t post_size(int c) const {
    int ci = comp_of.empty() ? -1 : comp_of[c];
    if (ci >= 0 && !rank.empty() && rank[ci] < size[c]) return rank[ci];
    return size[c];
  }
  // position of separator b in the adjacency list of separator a, or -1
  int64_t sadj_find(int a, int b) const {
    const int pa = sep_pos[a];
    const int32_t* lo = sadj_idx.data() + sadj_ptr[pa];
    const int32_t* hi = sadj_idx.data() + sadj_ptr[pa + 1];
    const int32_t* it = std::lower_bound(lo, hi, b);
    return (it == hi || *it != b) ? -1 : (int64_t)(it - sadj_idx.data());
  }
  int32_t find_pair(int a, int b) const {  // cluster indices, a <= b, both separators
    if (a == b) return pair_diag[sep_pos[a]];
    const int64_t e = sadj_find(a, b);
    return e < 0 ? -1 : sadj_pair[e];
  }
  // row of neighbour X inside the front of interior cluster I (m + offset)
  int32_t front_row(int I, int X) const {
    const int32_t* lo = adj_idx.data() + adj_ptr[I];
    const int32_t* hi = adj_idx.data() + adj_ptr[I + 1];
    const int64_t e = std::lower_bound(lo, hi, X) - adj_idx.data();
    return elim[elim_of[I]].m + nbr_off[e];
  }
};

struct Plan {
  Options opt;
  int64_t n = 0, n_nodes = 0;
  int pi = 1;
  std::vector<Partition> parts;            // partitions by level (index t-1)
  std::vector<Level> levels;
  std::vector<int64_t> perm;               // slot -> unknown
  std::vector<int64_t> csr_dst;            // level-1 arena offset per CSR entry (-1 = skip)
  double cmin[3] = {0, 0, 0}, cmax[3] = {0, 0, 0};
  int64_t max_node = 0;
};

// ---------------------------------------------------------------------------

// Which cells a scheme compresses (Sec. 5): Gen-All-All every box of the
// general partition; Nest-All-All every separator cell but single vertices;
// Nest-2-All and Nest-2-2 the cells of codimension one (faces in 3D, edges
// in 2D).
inline bool compressible(int type, int dim, int scheme) {
  if (scheme == SCHEME_GEN_ALL_ALL) return true;
  if (type == 0 || type == dim) return false;
  if (scheme == SCHEME_NEST_ALL_ALL) return true;
  return type == 1;
}

// Columns of N for compression d from its neighbours' sizes and `full`
// flags (Eq. 4.5; whole blocks for Nest-2-2 boundary cells and for the
// low-rank equivalent, which also drops the L_B^T Phi_B block and pads N
// with zero columns to at least s, so that a recorded rank up to s is a
// number of QR steps).
inline void comp_columns(CompDesc& d, CompNbr* nb, int pi, int compression) {
  d.self_cols = compression == 1 ? 0 : pi;
  int col = d.self_cols;
  for (int q = 0; q < d.nnb; ++q) {
    nb[q].col = col;
    col += nb[q].full ? nb[q].s_x : pi;
  }
  d.c = compression == 1 ? std::max(col, d.s) : col;
}

// Derive interiors, fronts, separator pairs, Schur lists and compression
// descriptors of a level whose clusters, sizes, slots and adjacency are set.
inline void build_level(Level& L, const Options& o, int pi, const Partition* part = nullptr) {
  const int nc = (int)L.cell.size();
  L.interiors.clear();
  L.seps.clear();
  L.sep_pos.assign(nc, -1);
  L.elim_of.assign(nc, -1);
  L.n_active = 0;
  for (int c = 0; c < nc; ++c) {
    L.n_active += L.size[c];
    if (L.top || L.type[c] == 0) {
      L.elim_of[c] = (int32_t)L.interiors.size();
      L.interiors.push_back(c);
    } else {
      L.sep_pos[c] = (int)L.seps.size();
      L.seps.push_back(c);
    }
  }
  const int ni = (int)L.interiors.size(), ns = (int)L.seps.size();
  // ---- interiors: fronts [I ; neighbours] -----------------------------------
  L.elim.assign(ni, ElimDesc{});
  L.nbr_off.assign(L.adj_idx.size(), 0);
  L.front_elems = 0;
  L.t_elems = 0;
  L.max_front_rows = 0;
  int64_t total_k = 0;
  for (int ii = 0; ii < ni; ++ii) {
    const int I = L.interiors[ii];
    ElimDesc& d = L.elim[ii];
    d.cluster = I;
    d.m = L.size[I];
    d.bw = d.m;
    d.pk_off = -1;
    int k = 0;
    for (int64_t e = L.adj_ptr[I]; e < L.adj_ptr[I + 1]; ++e) {
      const int X = L.adj_idx[e];
      if (L.sep_pos[X] < 0)
        throw std::runtime_error("two interiors are adjacent: the pattern couples nodes more than one grid step apart");
      L.nbr_off[e] = k;
      k += L.size[X];
    }
    d.k = k;
    d.front_off = L.front_elems;
    const int64_t R = (int64_t)d.m + k;
    L.front_elems += R * R;
    L.max_front_rows = std::max<int32_t>(L.max_front_rows, (int32_t)R);
    d.slot_off = L.slot_ptr[I];
    d.nslot_off = total_k;
    d.t_off = L.t_elems;
    L.t_elems += k;
    total_k += k;
  }
  L.nslots.resize(total_k);
  for (int ii = 0; ii < ni; ++ii) {
    const int I = L.interiors[ii];
    int64_t q = L.elim[ii].nslot_off;
    for (int64_t e = L.adj_ptr[I]; e < L.adj_ptr[I + 1]; ++e) {
      const int X = L.adj_idx[e];
      for (int64_t s = L.slot_ptr[X]; s < L.slot_ptr[X + 1]; ++s) L.nslots[q++] = L.slots[s];
    }
  }
  // ---- separators: post-elimination adjacency ------------------------------
  // sadj(a) = separators adjacent to a, plus every other neighbour of each
  // interior adjacent to a (the fill of Eq. 4.2).
  L.sadj_ptr.assign(ns + 1, 0);
  L.sadj_idx.clear();
  {
    std::vector<int32_t> stamp(nc, -1), buf;
    for (int p = 0; p < ns; ++p) {
      const int a = L.seps[p];
      buf.clear();
      stamp[a] = p;
      for (int64_t e = L.adj_ptr[a]; e < L.adj_ptr[a + 1]; ++e) {
        const int X = L.adj_idx[e];
        if (L.sep_pos[X] >= 0) {
          if (stamp[X] != p) {
            stamp[X] = p;
            buf.push_back(X);
          }
        } else {
          for (int64_t f = L.adj_ptr[X]; f < L.adj_ptr[X + 1]; ++f) {
            const int Y = L.adj_idx[f];
            if (stamp[Y] != p) {
              stamp[Y] = p;
              buf.push_back(Y);
            }
          }
        }
      }
      std::sort(buf.begin(), buf.end());
      L.sadj_idx.insert(L.sadj_idx.end(), buf.begin(), buf.end());
      L.sadj_ptr[p + 1] = (int64_t)L.sadj_idx.size();
    }
  }
  // pairs (a <= b): diagonal first, then upper neighbours ascending
  L.pairs.clear();
  L.pairs.reserve(ns + L.sadj_idx.size() / 2);
  L.sadj_pair.assign(L.sadj_idx.size(), -1);
  L.pair_diag.assign(ns, -1);
  L.blk_elems = 0;
  L.scratch_elems = 0;
  for (int p = 0; p < ns; ++p) {
    const int a = L.seps[p];
    auto add = [&](int b) {
      PairDesc d{};
      d.a = a;
      d.b = b;
      d.s_a = L.size[a];
      d.s_b = L.size[b];
      d.blk_off = L.blk_elems;
      L.blk_elems += (int64_t)d.s_a * d.s_b;
      d.scratch_off = L.scratch_elems;
      L.scratch_elems += 2 * (int64_t)d.s_a * d.s_b;
      d.ca = d.cb = -1;
      d.row_in_a = d.row_in_b = -1;
      L.pairs.push_back(d);
      return (int32_t)L.pairs.size() - 1;
    };
    L.pair_diag[p] = add(a);
    for (int64_t e = L.sadj_ptr[p]; e < L.sadj_ptr[p + 1]; ++e)
      if (L.sadj_idx[e] > a) L.sadj_pair[e] = add(L.sadj_idx[e]);
  }
  // Schur contributions, grouped per pair, interiors ascending (counting sort)
  {
    std::vector<int32_t> cnt(L.pairs.size() + 1, 0);
    std::vector<int32_t> pid_of;
    pid_of.reserve(L.adj_idx.size() * 4);
    for (int ii = 0; ii < ni; ++ii) {
      const int I = L.interiors[ii];
      for (int64_t x = L.adj_ptr[I]; x < L.adj_ptr[I + 1]; ++x)
        for (int64_t y = x; y < L.adj_ptr[I + 1]; ++y) {
          const int pid = L.find_pair(L.adj_idx[x], L.adj_idx[y]);
          pid_of.push_back(pid);
          ++cnt[pid + 1];
        }
    }
    for (size_t p = 0; p < L.pairs.size(); ++p) {
      L.pairs[p].c_ptr = cnt[p];
      L.pairs[p].c_cnt = cnt[p + 1];
      cnt[p + 1] += cnt[p];
    }
    L.schur.assign(pid_of.size(), SchurDesc{});
    L.schur_ii.assign(pid_of.size(), 0);
    L.schur_ex.assign(pid_of.size(), 0);
    L.schur_ey.assign(pid_of.size(), 0);
    std::vector<int32_t> cur(L.pairs.size());
    for (size_t p = 0; p < L.pairs.size(); ++p) cur[p] = L.pairs[p].c_ptr;
    size_t q = 0;
    for (int ii = 0; ii < ni; ++ii) {
      const int I = L.interiors[ii];
      const ElimDesc& e = L.elim[ii];
      const int64_t ld = (int64_t)e.m + e.k;
      for (int64_t x = L.adj_ptr[I]; x < L.adj_ptr[I + 1]; ++x)
        for (int64_t y = x; y < L.adj_ptr[I + 1]; ++y) {
          SchurDesc sd{};
          sd.src_ld = (int32_t)ld;
          sd.diag = x == y;
          sd.src_off = e.front_off + (e.m + L.nbr_off[y]) + (int64_t)(e.m + L.nbr_off[x]) * ld;
          const int32_t at = cur[pid_of[q++]]++;
          L.schur[at] = sd;
          L.schur_ii[at] = ii;
          L.schur_ex[at] = x;
          L.schur_ey[at] = y;
        }
    }
  }
  // ---- Phi per cluster ---------------------------------------------------------
  L.phi_off.assign(nc, 0);
  L.phi_elems = 0;
  for (int c = 0; c < nc; ++c) {
    L.phi_off[c] = L.phi_elems;
    L.phi_elems += (int64_t)L.size[c] * pi;
  }
  // ---- compressions --------------------------------------------------------------
  L.comp.clear();
  L.comp_nbr.clear();
  L.cnbr_x.clear();
  L.cnbr_pid.clear();
  L.cnbr_full.clear();
  L.comp_of.assign(nc, -1);
  L.cf_elems = L.n_elems = L.ltphi_elems = L.tau_elems = L.tb_elems = 0;
  L.max_cf_rows = L.max_c = L.max_s = 0;
  if (L.compress) {
    L.comp.reserve(ns);
    L.comp_nbr.reserve(L.sadj_idx.size());
    for (int p = 0; p < ns; ++p) {
      const int B = L.seps[p];
      if (!compressible(L.type[B], o.dim, o.scheme)) continue;
      CompDesc d{};
      d.cluster = B;
      d.s = L.size[B];
      d.nb_ptr = (int32_t)L.comp_nbr.size();
      d.nnb = (int32_t)(L.sadj_ptr[p + 1] - L.sadj_ptr[p]);
      int K = 0;
      for (int64_t e = L.sadj_ptr[p]; e < L.sadj_ptr[p + 1]; ++e) {
        const int X = L.sadj_idx[e];
        CompNbr nbx{};
        const int pid = X > B ? L.sadj_pair[e] : L.find_pair(X, B);
        nbx.blk_off = L.pairs[pid].blk_off;
        nbx.trans = X > B ? 1 : 0;
        nbx.s_x = L.size[X];
        nbx.phi_off = L.phi_off[X];
        nbx.row = d.s + K;
        nbx.full = o.compression == 1 ||
                   (o.scheme == SCHEME_NEST_2_2 && part && on_boundary(*part, L.cell[B], L.cell[X]));
        K += L.size[X];
        L.comp_nbr.push_back(nbx);
        L.cnbr_x.push_back(X);
        L.cnbr_pid.push_back(pid);
        L.cnbr_full.push_back((uint8_t)nbx.full);
      }
      d.K = K;
      comp_columns(d, L.comp_nbr.data() + d.nb_ptr, pi, o.compression);
      d.cf_off = L.cf_elems;
      L.cf_elems += (int64_t)(d.s + K) * d.s;
      d.n_off = L.n_elems;
      L.n_elems += (int64_t)d.s * d.c;
      d.ltphi_off = L.ltphi_elems;
      L.ltphi_elems += (int64_t)d.s * pi;
      d.tau_off = L.tau_elems;
      L.tau_elems += d.c;
      d.tb_off = L.tb_elems;
      L.tb_elems += (int64_t)d.s * d.s;
      d.phi_off = L.phi_off[B];
      d.slot_off = L.slot_ptr[B];
      d.blk_diag = L.pairs[L.pair_diag[p]].blk_off;
      L.comp_of[B] = (int32_t)L.comp.size();
      L.max_cf_rows = std::max<int32_t>(L.max_cf_rows, d.s + K);
      L.max_c = std::max<int32_t>(L.max_c, d.c);
      L.max_s = std::max<int32_t>(L.max_s, d.s);
      L.comp.push_back(d);
    }
  }
  // pair descriptors: compression indices and rows inside the fronts
  L.pair_rowa.assign(L.pairs.size(), -1);
  L.pair_rowb.assign(L.pairs.size(), -1);
  for (size_t p = 0; p < L.pairs.size(); ++p) {
    PairDesc& pd = L.pairs[p];
    pd.ca = L.comp_of[pd.a];
    pd.cb = L.comp_of[pd.b];
    if (pd.a != pd.b) {
      if (pd.ca >= 0) {
        const CompDesc& d = L.comp[pd.ca];
        const int64_t e = L.sadj_find(pd.a, pd.b);
        L.pair_rowa[p] = (int32_t)(d.nb_ptr + (e - L.sadj_ptr[L.sep_pos[pd.a]]));
        pd.row_in_a = L.comp_nbr[L.pair_rowa[p]].row;
      }
      if (pd.cb >= 0) {
        const CompDesc& d = L.comp[pd.cb];
        const int64_t e = L.sadj_find(pd.b, pd.a);
        L.pair_rowb[p] = (int32_t)(d.nb_ptr + (e - L.sadj_ptr[L.sep_pos[pd.b]]));
        pd.row_in_b = L.comp_nbr[L.pair_rowb[p]].row;
      }
    }
  }
  // apply: separator accumulation lists (counting sort, interiors ascending)
  {
    std::vector<int32_t> cnt(ns + 1, 0);
    for (int ii = 0; ii < ni; ++ii) {
      const int I = L.interiors[ii];
      for (int64_t e = L.adj_ptr[I]; e < L.adj_ptr[I + 1]; ++e) ++cnt[L.sep_pos[L.adj_idx[e]] + 1];
    }
    std::vector<int32_t> start(ns + 1, 0);
    for (int p = 0; p < ns; ++p) start[p + 1] = start[p] + cnt[p + 1];
    std::vector<int64_t> flat(start[ns]), flat_e(start[ns]);
    std::vector<int32_t> flat_ii(start[ns]);
    std::vector<int32_t> cur(start.begin(), start.end() - 1);
    for (int ii = 0; ii < ni; ++ii) {
      const int I = L.interiors[ii];
      for (int64_t e = L.adj_ptr[I]; e < L.adj_ptr[I + 1]; ++e) {
        const int32_t at = cur[L.sep_pos[L.adj_idx[e]]]++;
        flat[at] = L.elim[ii].t_off + L.nbr_off[e];
        flat_ii[at] = ii;
        flat_e[at] = e;
      }
    }
    L.sepacc.clear();
    L.sepacc_src.clear();
    L.sepacc_src.reserve(flat.size());
    L.sacc_p.clear();
    L.sacc_ii.clear();
    L.sacc_e.clear();
    for (int p = 0; p < ns; ++p) {
      if (start[p + 1] == start[p]) continue;
      SepAcc sa{};
      sa.slot_off = L.slot_ptr[L.seps[p]];
      sa.s = L.size[L.seps[p]];
      sa.c_ptr = (int32_t)L.sepacc_src.size();
      sa.c_cnt = start[p + 1] - start[p];
      L.sepacc_src.insert(L.sepacc_src.end(), flat.begin() + start[p], flat.begin() + start[p + 1]);
      L.sacc_ii.insert(L.sacc_ii.end(), flat_ii.begin() + start[p], flat_ii.begin() + start[p + 1]);
      L.sacc_e.insert(L.sacc_e.end(), flat_e.begin() + start[p], flat_e.begin() + start[p + 1]);
      L.sepacc.push_back(sa);
      L.sacc_p.push_back(p);
    }
  }
  L.rank.clear();
  L.capply.clear();
}

// Every size-dependent field of a level whose structure build_level has
// recorded, from its current cluster sizes: the same values build_level
// gives for these sizes, without its adjacency searches and sorts.
inline void build_offsets(Level& L, int pi, int compression) {
  const int nc = (int)L.cell.size();
  L.n_active = 0;
  for (int c = 0; c < nc; ++c) L.n_active += L.size[c];
  // interiors
  L.front_elems = 0;
  L.t_elems = 0;
  L.max_front_rows = 0;
  int64_t total_k = 0;
  for (size_t ii = 0; ii < L.interiors.size(); ++ii) {
    const int I = L.interiors[ii];
    ElimDesc& d = L.elim[ii];
    d.m = L.size[I];
    d.bw = d.m;
    d.pk_off = -1;
    int k = 0;
    for (int64_t e = L.adj_ptr[I]; e < L.adj_ptr[I + 1]; ++e) {
      L.nbr_off[e] = k;
      k += L.size[L.adj_idx[e]];
    }
    d.k = k;
    d.front_off = L.front_elems;
    const int64_t R = (int64_t)d.m + k;
    L.front_elems += R * R;
    L.max_front_rows = std::max<int32_t>(L.max_front_rows, (int32_t)R);
    d.slot_off = L.slot_ptr[I];
    d.nslot_off = total_k;
    d.t_off = L.t_elems;
    L.t_elems += k;
    total_k += k;
  }
  L.nslots.resize(total_k);
  for (size_t ii = 0; ii < L.interiors.size(); ++ii) {
    const int I = L.interiors[ii];
    int64_t q = L.elim[ii].nslot_off;
    for (int64_t e = L.adj_ptr[I]; e < L.adj_ptr[I + 1]; ++e) {
      const int X = L.adj_idx[e];
      for (int64_t s = L.slot_ptr[X]; s < L.slot_ptr[X + 1]; ++s) L.nslots[q++] = L.slots[s];
    }
  }
  // pair blocks, in pair order
  L.blk_elems = 0;
  L.scratch_elems = 0;
  for (PairDesc& d : L.pairs) {
    d.s_a = L.size[d.a];
    d.s_b = L.size[d.b];
    d.blk_off = L.blk_elems;
    L.blk_elems += (int64_t)d.s_a * d.s_b;
    d.scratch_off = L.scratch_elems;
    L.scratch_elems += 2 * (int64_t)d.s_a * d.s_b;
  }
  // Schur sources
  for (size_t q = 0; q < L.schur.size(); ++q) {
    const ElimDesc& e = L.elim[L.schur_ii[q]];
    const int64_t ld = (int64_t)e.m + e.k;
    L.schur[q].src_ld = (int32_t)ld;
    L.schur[q].src_off = e.front_off + (e.m + L.nbr_off[L.schur_ey[q]]) + (e.m + L.nbr_off[L.schur_ex[q]]) * ld;
  }
  // Phi per cluster
  L.phi_elems = 0;
  for (int c = 0; c < nc; ++c) {
    L.phi_off[c] = L.phi_elems;
    L.phi_elems += (int64_t)L.size[c] * pi;
  }
  // compressions
  L.cf_elems = L.n_elems = L.ltphi_elems = L.tau_elems = L.tb_elems = 0;
  L.max_cf_rows = L.max_c = L.max_s = 0;
  for (CompDesc& d : L.comp) {
    const int B = d.cluster;
    d.s = L.size[B];
    int K = 0;
    for (int q = 0; q < d.nnb; ++q) {
      const int at = d.nb_ptr + q;
      CompNbr& nbx = L.comp_nbr[at];
      const int X = L.cnbr_x[at];
      nbx.blk_off = L.pairs[L.cnbr_pid[at]].blk_off;
      nbx.s_x = L.size[X];
      nbx.phi_off = L.phi_off[X];
      nbx.row = d.s + K;
      nbx.full = L.cnbr_full[at];
      K += L.size[X];
    }
    d.K = K;
    comp_columns(d, L.comp_nbr.data() + d.nb_ptr, pi, compression);
    d.cf_off = L.cf_elems;
    L.cf_elems += (int64_t)(d.s + K) * d.s;
    d.n_off = L.n_elems;
    L.n_elems += (int64_t)d.s * d.c;
    d.ltphi_off = L.ltphi_elems;
    L.ltphi_elems += (int64_t)d.s * pi;
    d.tau_off = L.tau_elems;
    L.tau_elems += d.c;
    d.tb_off = L.tb_elems;
    L.tb_elems += (int64_t)d.s * d.s;
    d.phi_off = L.phi_off[B];
    d.slot_off = L.slot_ptr[B];
    d.blk_diag = L.pairs[L.pair_diag[L.sep_pos[B]]].blk_off;
    L.max_cf_rows = std::max<int32_t>(L.max_cf_rows, d.s + K);
    L.max_c = std::max<int32_t>(L.max_c, d.c);
    L.max_s = std::max<int32_t>(L.max_s, d.s);
  }
  for (size_t p = 0; p < L.pairs.size(); ++p) {
    if (L.pair_rowa[p] >= 0) L.pairs[p].row_in_a = L.comp_nbr[L.pair_rowa[p]].row;
    if (L.pair_rowb[p] >= 0) L.pairs[p].row_in_b = L.comp_nbr[L.pair_rowb[p]].row;
  }
  // apply: separator accumulation
  for (size_t a = 0; a < L.sepacc.size(); ++a) {
    const int B = L.seps[L.sacc_p[a]];
    L.sepacc[a].slot_off = L.slot_ptr[B];
    L.sepacc[a].s = L.size[B];
  }
  for (size_t j = 0; j < L.sepacc_src.size(); ++j)
    L.sepacc_src[j] = L.elim[L.sacc_ii[j]].t_off + L.nbr_off[L.sacc_e[j]];
  L.rank.clear();
  L.capply.clear();
}

// Bounds check of every descriptor of a level against its buffers; throws
// on the first violation so that no kernel is launched on a bad table.
inline void validate_level(const Level& L, int64_t n, int pi) {
  auto req = [](bool ok, const char* what) {
    if (!ok) throw std::runtime_error(std::string("plan bounds check failed: ") + what);
  };
  const int64_t arena = L.front_elems + L.blk_elems;
  const int64_t nsl = (int64_t)L.slots.size(), nns = (int64_t)L.nslots.size();
  // slot values above level 1 are copies of checked level-1 slots
  if (L.t == 1) {
    for (int32_t v : L.slots) req(v >= 0 && v < n, "slot out of range");
    for (int32_t v : L.nslots) req(v >= 0 && v < n, "neighbour slot out of range");
  }
  for (const auto& e : L.elim) {
    int64_t R = (int64_t)e.m + e.k;
    req(e.m >= 0 && e.k >= 0 && e.front_off >= 0 && e.front_off + R * R <= L.front_elems, "front extent");
    req(e.slot_off >= 0 && e.slot_off + e.m <= nsl, "interior slots");
    req(e.nslot_off >= 0 && e.nslot_off + e.k <= nns, "interior neighbour slots");
    req(e.t_off >= 0 && e.t_off + e.k <= L.t_elems, "apply scratch");
  }
  for (const auto& p : L.pairs) {
    int64_t ab = (int64_t)p.s_a * p.s_b;
    req(p.s_a > 0 && p.s_b > 0, "empty pair block");
    req(p.blk_off >= 0 && p.blk_off + ab <= L.blk_elems, "pair block extent");
    req(p.scratch_off >= 0 && p.scratch_off + 2 * ab <= L.scratch_elems, "pair scratch extent");
    req(p.c_ptr >= 0 && p.c_ptr + p.c_cnt <= (int64_t)L.schur.size(), "schur list");
    req(p.ca < (int)L.comp.size() && p.cb < (int)L.comp.size(), "pair compression index");
    if (p.a != p.b && p.ca >= 0)
      req(p.row_in_a >= L.comp[p.ca].s && p.row_in_a + p.s_b <= L.comp[p.ca].s + L.comp[p.ca].K, "row in a");
    if (p.a != p.b && p.cb >= 0)
      req(p.row_in_b >= L.comp[p.cb].s && p.row_in_b + p.s_a <= L.comp[p.cb].s + L.comp[p.cb].K, "row in b");
    for (int c = 0; c < p.c_cnt; ++c) {
      const SchurDesc& s = L.schur[p.c_ptr + c];
      int64_t last = s.diag ? s.src_off + (p.s_a - 1) + (int64_t)(p.s_a - 1) * s.src_ld
                            : s.src_off + (p.s_b - 1) + (int64_t)(p.s_a - 1) * s.src_ld;
      req(s.src_off >= 0 && last < L.front_elems, "schur source extent");
    }
  }
  for (const auto& d : L.comp) {
    req(d.s > 0 && d.cf_off >= 0 && d.cf_off + (int64_t)(d.s + d.K) * d.s <= L.cf_elems, "compression front");
    req(d.n_off >= 0 && d.n_off + (int64_t)d.s * d.c <= L.n_elems, "N buffer");
    req(d.phi_off >= 0 && d.phi_off + (int64_t)d.s * pi <= L.phi_elems, "Phi_B");
    req(d.ltphi_off >= 0 && d.ltphi_off + (int64_t)d.s * pi <= L.ltphi_elems, "LtPhi");
    req(d.tau_off >= 0 && d.tau_off + d.c <= L.tau_elems, "tau");
    req(d.tb_off >= 0 && d.tb_off + (int64_t)d.s * d.s <= L.tb_elems, "T_B slot");
    req(d.slot_off >= 0 && d.slot_off + d.s <= nsl, "compression slots");
    req(d.blk_diag >= 0 && d.blk_diag + (int64_t)d.s * d.s <= L.blk_elems, "diagonal block");
    req(d.nb_ptr >= 0 && d.nb_ptr + d.nnb <= (int64_t)L.comp_nbr.size(), "neighbour list");
    int K = 0;
    for (int q = 0; q < d.nnb; ++q) {
      const CompNbr& x = L.comp_nbr[d.nb_ptr + q];
      req(x.blk_off >= 0 && x.blk_off + (int64_t)d.s * x.s_x <= L.blk_elems, "neighbour block");
      req(x.phi_off >= 0 && x.phi_off + (int64_t)x.s_x * pi <= L.phi_elems, "neighbour Phi");
      req(x.row == d.s + K, "neighbour row");
      req(x.col >= d.self_cols && x.col + (x.full ? x.s_x : pi) <= d.c, "neighbour columns of N");
      req(q == 0 || x.col == L.comp_nbr[d.nb_ptr + q - 1].col + (L.comp_nbr[d.nb_ptr + q - 1].full
                                                                    ? L.comp_nbr[d.nb_ptr + q - 1].s_x : pi),
          "neighbour columns in order");
      K += x.s_x;
    }
    req(K == d.K, "neighbour total");
    req(d.self_cols == 0 || d.self_cols == pi, "self columns of N");
    req(d.c >= d.self_cols && d.c >= 1, "columns of N");
  }
  for (const auto& a : L.sepacc) {
    req(a.slot_off >= 0 && a.slot_off + a.s <= nsl, "separator slots");
    req(a.c_ptr >= 0 && a.c_ptr + a.c_cnt <= (int64_t)L.sepacc_src.size(), "accumulation list");
    for (int c = 0; c < a.c_cnt; ++c) {
      int64_t v = L.sepacc_src[a.c_ptr + c];
      req(v >= 0 && v + a.s <= L.t_elems, "accumulation source");
    }
  }
  req((int64_t)L.phi_off.size() == (int64_t)L.cell.size(), "phi offsets");
  (void)arena;
}

inline void validate_copies(const std::vector<CopyDesc>& v, int64_t src_elems, int64_t dst_elems) {
  for (const auto& c : v) {
    if (c.rows <= 0 || c.cols <= 0) throw std::runtime_error("plan bounds check failed: empty copy");
    int64_t s_last = c.src_off + (c.rows - 1) + (int64_t)(c.cols - 1) * c.src_ld;
    int64_t d_last = c.mode == 0 ? c.dst_off + (c.rows - 1) + (int64_t)(c.cols - 1) * c.dst_ld
                                 : c.dst_off + (c.cols - 1) + (int64_t)(c.rows - 1) * c.dst_ld;
    if (c.src_off < 0 || s_last >= src_elems || c.dst_off < 0 || d_last >= dst_elems)
      throw std::runtime_error("plan bounds check failed: copy extent");
  }
}

// Level 1 from the CSR pattern.
inline void plan_level1(Plan& P, const int64_t* row_ptr, const int32_t* col_idx) {
  const Options& o = P.opt;
  Partition part = make_partition(o, o.leaf);
  P.parts.clear();
  P.parts.push_back(part);
  const int64_t nn = P.n_nodes;
  const int dpn = o.dpn;
  // cell of every node
  std::vector<int64_t> cell_of_node(nn);
  int gx = o.grid[0], gy = o.dim >= 2 ? o.grid[1] : 1;
  for (int64_t v = 0; v < nn; ++v) {
    int ix = (int)(v % gx), iy = (int)((v / gx) % gy), iz = (int)(v / ((int64_t)gx * gy));
    cell_of_node[v] = part.cell_of(ix, iy, o.dim >= 3 ? iz : 0);
  }
  // counting sort by cell; clusters = non-empty cells ascending
  std::vector<int64_t> cnt(part.ncells + 1, 0);
  for (int64_t v = 0; v < nn; ++v) cnt[cell_of_node[v] + 1] += dpn;
  std::vector<int32_t> cluster_of_cell(part.ncells, -1);
  Level L;
  L.t = 1;
  L.top = part.is_root;
  L.compress = o.compress && o.compress_from_level <= 1 && !L.top;
  for (int64_t c = 0; c < part.ncells; ++c)
    if (cnt[c + 1] > 0) {
      cluster_of_cell[c] = (int32_t)L.cell.size();
      L.cell.push_back(c);
      L.type.push_back(part.type_of(c));
      L.size.push_back((int32_t)cnt[c + 1]);
    }
  for (int64_t c = 0; c < part.ncells; ++c) cnt[c + 1] += cnt[c];
  P.perm.assign(P.n, 0);
  std::vector<int32_t> cl_of(P.n), loc_of(P.n);
  std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
  for (int64_t v = 0; v < nn; ++v)
    for (int c = 0; c < dpn; ++c) {
      int64_t dof = v * dpn + c;
      int64_t cc = cell_of_node[v];
      int64_t s = pos[cc]++;
      P.perm[s] = dof;
      cl_of[dof] = cluster_of_cell[cc];
      loc_of[dof] = (int32_t)(s - cnt[cc]);
    }
  const int nc = (int)L.cell.size();
  L.slot_ptr.assign(nc + 1, 0);
  for (int c = 0; c < nc; ++c) L.slot_ptr[c + 1] = L.slot_ptr[c] + L.size[c];
  L.slots.resize(P.n);
  for (int64_t s = 0; s < P.n; ++s) L.slots[s] = (int32_t)s;
  // adjacency from the pattern; check the 3^dim stencil assumption
  std::vector<std::vector<int32_t>> adj(nc);
  for (int64_t i = 0; i < P.n; ++i) {
    int ci = cl_of[i];
    int64_t ni = i / dpn;
    int ix = (int)(ni % gx), iy = (int)((ni / gx) % gy), iz = (int)(ni / ((int64_t)gx * gy));
    for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      int64_t j = col_idx[e];
      if (j < 0 || j >= P.n) throw std::runtime_error("column index out of range");
      int64_t nj = j / dpn;
      int jx = (int)(nj % gx), jy = (int)((nj / gx) % gy), jz = (int)(nj / ((int64_t)gx * gy));
      if (std::abs(ix - jx) > 1 || std::abs(iy - jy) > 1 || std::abs(iz - jz) > 1)
        throw std::runtime_error("pattern couples grid nodes more than one step apart");
      int cj = cl_of[j];
      if (cj != ci) adj[ci].push_back(cj);
    }
  }
  L.adj_ptr.assign(nc + 1, 0);
  L.adj_idx.clear();
  for (int c = 0; c < nc; ++c) {
    auto& v = adj[c];
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    L.adj_idx.insert(L.adj_idx.end(), v.begin(), v.end());
    L.adj_ptr[c + 1] = (int64_t)L.adj_idx.size();
  }
  build_level(L, o, P.pi, &part);
  P.max_node = 0;
  for (int c = 0; c < nc; ++c) P.max_node = std::max<int64_t>(P.max_node, L.size[c]);
  // CSR fill destinations
  const int64_t nnz = row_ptr[P.n];
  P.csr_dst.assign(nnz, -1);
  const std::vector<int32_t>& elim_of = L.elim_of;
  for (auto& d : L.elim) d.bw = 0;
  for (int64_t i = 0; i < P.n; ++i) {
    int ci = cl_of[i], li = loc_of[i];
    for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      int64_t j = col_idx[e];
      int cj = cl_of[j], lj = loc_of[j];
      if (elim_of[ci] >= 0) {
        const ElimDesc& d = L.elim[elim_of[ci]];
        int64_t ld = (int64_t)d.m + d.k;
        if (cj == ci) {
          P.csr_dst[e] = d.front_off + li + (int64_t)lj * ld;
          L.elim[elim_of[ci]].bw = std::max(L.elim[elim_of[ci]].bw, std::abs(li - lj));
        } else {
          int64_t row = L.front_row(ci, cj) + lj;
          P.csr_dst[e] = d.front_off + row + (int64_t)li * ld;
        }
      } else if (elim_of[cj] >= 0) {
        // separator row, interior column: written from the symmetric entry
      } else if (ci <= cj) {
        int pid = L.find_pair(ci, cj);
        const PairDesc& pd = L.pairs[pid];
        P.csr_dst[e] = L.front_elems + pd.blk_off + li + (int64_t)lj * pd.s_a;
      }
    }
  }
  for (int64_t d : P.csr_dst)
    if (d >= L.front_elems + L.blk_elems) throw std::runtime_error("plan bounds check failed: CSR fill");
  validate_level(L, P.n, P.pi);
  P.levels.clear();
  P.levels.push_back(std::move(L));
}

// Copy maps from level C to the next level N: the coarse part (ld s_a) of
// every level-C pair block into N's storage (where N.cp_kind says), and the
// Phi rows of every surviving separator into its father's Phi.  `father`
// and `loc`: each separator's father in N and its first row there.
inline void emit_copy_maps(const Level& C, const Level& N, const std::vector<int32_t>& father,
                           const std::vector<int32_t>& loc, int pi, std::vector<CopyDesc>& blk_map,
                           std::vector<CopyDesc>& phi_map) {
  blk_map.clear();
  phi_map.clear();
  blk_map.reserve(2 * C.pairs.size());
  for (size_t q = 0; q < C.pairs.size(); ++q) {
    const PairDesc& pd = C.pairs[q];
    const int pa = C.sep_pos[pd.a], pb = C.sep_pos[pd.b];
    const int ra = C.post_size(pd.a), rb = C.post_size(pd.b);
    if (ra == 0 || rb == 0) continue;
    const int oa = loc[pa], ob = loc[pb];
    CopyDesc cd{};
    cd.src_off = C.front_elems + pd.blk_off;
    cd.src_ld = pd.s_a;
    cd.rows = ra;
    cd.cols = rb;
    const int kind = N.cp_kind[q], tg = N.cp_tgt[q];
    if (kind == 0 || kind == 1) {
      int64_t base, ld;
      if (kind == 0) {
        const ElimDesc& e = N.elim[tg];
        base = e.front_off;
        ld = (int64_t)e.m + e.k;
      } else {
        const PairDesc& p2 = N.pairs[tg];
        base = N.front_elems + p2.blk_off;
        ld = p2.s_a;
      }
      cd.dst_ld = (int32_t)ld;
      cd.mode = 0;
      cd.dst_off = base + oa + (int64_t)ob * ld;
      blk_map.push_back(cd);
      if (pd.a != pd.b) {
        cd.mode = 1;
        cd.dst_off = base + ob + (int64_t)oa * ld;
        blk_map.push_back(cd);
      }
    } else if (kind == 2 || kind == 3) {
      const ElimDesc& e = N.elim[tg];
      const int64_t ld = (int64_t)e.m + e.k;
      const int64_t row = e.m + N.nbr_off[N.cp_e[q]];
      cd.dst_ld = (int32_t)ld;
      if (kind == 2) {
        cd.mode = 1;
        cd.dst_off = e.front_off + (row + ob) + (int64_t)oa * ld;
      } else {
        cd.mode = 0;
        cd.dst_off = e.front_off + (row + oa) + (int64_t)ob * ld;
      }
      blk_map.push_back(cd);
    } else {
      const PairDesc& p2 = N.pairs[tg];
      cd.dst_ld = p2.s_a;
      if (kind == 4) {
        cd.mode = 0;
        cd.dst_off = N.front_elems + p2.blk_off + oa + (int64_t)ob * p2.s_a;
      } else {
        cd.mode = 1;
        cd.dst_off = N.front_elems + p2.blk_off + ob + (int64_t)oa * p2.s_a;
      }
      blk_map.push_back(cd);
    }
  }
  if (!N.top) {
    phi_map.reserve(C.seps.size());
    for (size_t p = 0; p < C.seps.size(); ++p) {
      const int a = C.seps[p];
      const int r = C.post_size(a);
      if (r == 0) continue;
      CopyDesc cd{};
      cd.src_off = C.phi_off[a];
      cd.src_ld = C.size[a];
      cd.rows = r;
      cd.cols = pi;
      cd.mode = 0;
      const int D = father[p];
      cd.dst_ld = N.size[D];
      cd.dst_off = N.phi_off[D] + loc[p];
      phi_map.push_back(cd);
    }
  }
}

// The structure-only coarsening tables of the pair blocks and separators of
// level C into level N (see CoarsenPair).
inline void coarsen_tables(const Level& C, const Level& N, std::vector<CoarsenPair>& cp, std::vector<CoarsenSep>& cs) {
  cp.resize(C.pairs.size());
  for (size_t q = 0; q < C.pairs.size(); ++q) {
    CoarsenPair& x = cp[q];
    x.kind = N.cp_kind[q];
    x.tgt = N.cp_tgt[q];
    x.e = N.cp_e[q];
    x.pa = C.sep_pos[C.pairs[q].a];
    x.pb = C.sep_pos[C.pairs[q].b];
  }
  cs.resize(C.seps.size());
  for (size_t p = 0; p < C.seps.size(); ++p) {
    cs[p].cluster = C.seps[p];
    cs[p].ci = C.comp_of.empty() ? -1 : C.comp_of[C.seps[p]];
  }
}

// Next level from the current one once its ranks are known (Secs. 4.3-4.4).
// Returns the copy maps for the pair blocks and for Phi.
inline void plan_next_level(Plan& P, std::vector<CopyDesc>& blk_map, std::vector<CopyDesc>& phi_map,
                            bool emit = true) {
  const Options& o = P.opt;
  Level& C = P.levels.back();
  C.planned_rank = C.rank;
  const Partition& lo = P.parts.back();
  Partition hi = make_partition(o, lo.d * 2);
  const int cs = (int)C.seps.size();
  // surviving clusters: the separators, with their post-compression sizes
  std::vector<int64_t> fcell(cs);
  for (int p = 0; p < cs; ++p) fcell[p] = father_cell(lo, hi, C.cell[C.seps[p]]);
  // father cells present, ascending (dense marking over the coarser cells)
  std::vector<int32_t> rank_of_cell(hi.ncells, -1);
  for (int p = 0; p < cs; ++p) rank_of_cell[fcell[p]] = 0;
  std::vector<int64_t> uniq;
  for (int64_t c = 0; c < hi.ncells; ++c)
    if (rank_of_cell[c] == 0) {
      rank_of_cell[c] = (int32_t)uniq.size();
      uniq.push_back(c);
    }
  Level N;
  N.t = C.t + 1;
  const int nc = (int)uniq.size();
  std::vector<int32_t> father(cs);
  for (int p = 0; p < cs; ++p) father[p] = rank_of_cell[fcell[p]];
  N.cell = uniq;
  N.type.resize(nc);
  for (int c = 0; c < nc; ++c) N.type[c] = hi.type_of(uniq[c]);
  N.size.assign(nc, 0);
  std::vector<int32_t> loc(cs);
  for (int p = 0; p < cs; ++p) {     // seps ascending: children in order
    loc[p] = N.size[father[p]];
    N.size[father[p]] += C.post_size(C.seps[p]);
  }
  int64_t n_active = 0, biggest = 0;
  for (int c = 0; c < nc; ++c) {
    n_active += N.size[c];
    biggest = std::max<int64_t>(biggest, N.size[c]);
  }
  P.max_node = std::max<int64_t>(P.max_node, biggest);
  bool top = hi.is_root || (o.stop_rule == 1 && n_active < P.max_node);
  N.from_father = father;
  N.from_nfathers = nc;
  N.from_merged = top && nc > 1;
  if (top && nc > 1) {
    // merge every cluster of the new partition into one, ascending cell id
    std::vector<int32_t> base(nc, 0);
    for (int c = 1; c < nc; ++c) base[c] = base[c - 1] + N.size[c - 1];
    for (int p = 0; p < cs; ++p) loc[p] += base[father[p]];
    for (auto& f : father) f = 0;
    N.cell = {uniq[0]};
    N.type = {0};
    N.size = {(int32_t)n_active};
  }
  N.top = top;
  const int nc2 = (int)N.cell.size();
  N.compress = !top && o.compress && N.t >= o.compress_from_level;
  // slots: concatenation of the children's first post-size slots
  N.slot_ptr.assign(nc2 + 1, 0);
  for (int c = 0; c < nc2; ++c) N.slot_ptr[c + 1] = N.slot_ptr[c] + N.size[c];
  N.slots.assign(N.slot_ptr[nc2], 0);
  for (int p = 0; p < cs; ++p) {
    const int a = C.seps[p];
    const int r = C.post_size(a);
    std::copy(C.slots.begin() + C.slot_ptr[a], C.slots.begin() + C.slot_ptr[a] + r,
              N.slots.begin() + N.slot_ptr[father[p]] + loc[p]);
  }
  // children grouped by father (ascending)
  std::vector<int32_t> ch_ptr(nc2 + 1, 0), ch(cs);
  for (int p = 0; p < cs; ++p) ++ch_ptr[father[p] + 1];
  for (int c = 0; c < nc2; ++c) ch_ptr[c + 1] += ch_ptr[c];
  {
    std::vector<int32_t> cur(ch_ptr.begin(), ch_ptr.end() - 1);
    for (int p = 0; p < cs; ++p) ch[cur[father[p]]++] = p;
  }
  // adjacency: fathers of adjacent separators
  N.adj_ptr.assign(nc2 + 1, 0);
  N.adj_idx.clear();
  {
    std::vector<int32_t> stamp(nc2, -1), buf;
    for (int fa = 0; fa < nc2; ++fa) {
      buf.clear();
      stamp[fa] = fa;
      for (int q = ch_ptr[fa]; q < ch_ptr[fa + 1]; ++q) {
        const int p = ch[q];
        for (int64_t e = C.sadj_ptr[p]; e < C.sadj_ptr[p + 1]; ++e) {
          const int fb = father[C.sep_pos[C.sadj_idx[e]]];
          if (stamp[fb] != fa) {
            stamp[fb] = fa;
            buf.push_back(fb);
          }
        }
      }
      std::sort(buf.begin(), buf.end());
      N.adj_idx.insert(N.adj_idx.end(), buf.begin(), buf.end());
      N.adj_ptr[fa + 1] = (int64_t)N.adj_idx.size();
    }
  }
  build_level(N, o, P.pi, &hi);
  // where each level-C pair block goes (by the new level's structure)
  const int ncp = (int)C.pairs.size();
  N.cp_kind.assign(ncp, -1);
  N.cp_tgt.assign(ncp, -1);
  N.cp_e.assign(ncp, -1);
  auto adj_entry = [&](int I, int X) {
    const int32_t* lo = N.adj_idx.data() + N.adj_ptr[I];
    const int32_t* hi2 = N.adj_idx.data() + N.adj_ptr[I + 1];
    const int32_t* it = std::lower_bound(lo, hi2, X);
    if (it == hi2 || *it != X) throw std::runtime_error("plan check failed: neighbour not adjacent");
    return (int64_t)(it - N.adj_idx.data());
  };
  auto pair_of = [&](int a, int b) {
    const int32_t q = N.find_pair(a, b);
    if (q < 0) throw std::runtime_error("plan check failed: missing pair block");
    return q;
  };
  for (int q = 0; q < ncp; ++q) {
    const PairDesc& pd = C.pairs[q];
    const int Da = father[C.sep_pos[pd.a]], Db = father[C.sep_pos[pd.b]];
    if (Da == Db) {
      if (N.elim_of[Da] >= 0) {
        N.cp_kind[q] = 0;
        N.cp_tgt[q] = N.elim_of[Da];
      } else {
        N.cp_kind[q] = 1;
        N.cp_tgt[q] = N.pair_diag[N.sep_pos[Da]];
      }
    } else if (N.elim_of[Da] >= 0) {
      N.cp_kind[q] = 2;
      N.cp_tgt[q] = N.elim_of[Da];
      N.cp_e[q] = adj_entry(Da, Db);
    } else if (N.elim_of[Db] >= 0) {
      N.cp_kind[q] = 3;
      N.cp_tgt[q] = N.elim_of[Db];
      N.cp_e[q] = adj_entry(Db, Da);
    } else if (Da < Db) {
      N.cp_kind[q] = 4;
      N.cp_tgt[q] = pair_of(Da, Db);
    } else {
      N.cp_kind[q] = 5;
      N.cp_tgt[q] = pair_of(Db, Da);
    }
  }
  N.can_update = true;
  N.cp_father = father;
  N.cp_loc = loc;
  if (!emit) {
    validate_level(N, P.n, P.pi);
    P.parts.push_back(hi);
    P.levels.push_back(std::move(N));
    return;
  }
  emit_copy_maps(C, N, father, loc, P.pi, blk_map, phi_map);
  validate_level(N, P.n, P.pi);
  validate_copies(blk_map, C.front_elems + C.blk_elems, N.front_elems + N.blk_elems);
  validate_copies(phi_map, C.phi_elems, N.phi_elems);
  P.parts.push_back(hi);
  P.levels.push_back(std::move(N));
}

// Whether update_next_level can take the recorded next level of level li:
// the rank-dependent top rule is off and that level was planned before for
// this level's clusters and pairs.
inline bool can_update_next_level(const Plan& P, size_t li) {
  if (P.opt.stop_rule != 0 || li + 1 >= P.levels.size()) return false;
  const Level& C = P.levels[li];
  const Level& N = P.levels[li + 1];
  return N.can_update && N.from_father.size() == C.seps.size() && N.cp_kind.size() == C.pairs.size();
}

// The next level re-planned in place for new ranks of level li: its
// clusters, adjacency, pairs and the order of every list depend only on the
// partition (with the fixed top rule), so only the sizes, slots and the
// offsets derived from them change.  Gives the same level and copy maps as
// plan_next_level for these ranks; false when the recorded structure cannot
// be used (no next level yet, or the rank-dependent top rule).
inline bool update_next_level(Plan& P, size_t li, std::vector<CopyDesc>& blk_map,
                              std::vector<CopyDesc>& phi_map, bool emit = true) {
  if (P.opt.stop_rule != 0 || li + 1 >= P.levels.size()) return false;
  Level& C = P.levels[li];
  Level& N = P.levels[li + 1];
  const int cs = (int)C.seps.size();
  if (!N.can_update || (int)N.from_father.size() != cs || N.cp_kind.size() != C.pairs.size()) return false;
  C.planned_rank = C.rank;
  const int nf = N.from_nfathers;
  std::vector<int32_t> loc(cs), father(cs), fsize(nf, 0);
  for (int p = 0; p < cs; ++p) {
    loc[p] = fsize[N.from_father[p]];
    fsize[N.from_father[p]] += C.post_size(C.seps[p]);
  }
  int64_t n_active = 0, biggest = 0;
  for (int c = 0; c < nf; ++c) {
    n_active += fsize[c];
    biggest = std::max<int64_t>(biggest, fsize[c]);
  }
  P.max_node = std::max<int64_t>(P.max_node, biggest);
  if (N.from_merged) {
    std::vector<int32_t> base(nf, 0);
    for (int c = 1; c < nf; ++c) base[c] = base[c - 1] + fsize[c - 1];
    for (int p = 0; p < cs; ++p) {
      loc[p] += base[N.from_father[p]];
      father[p] = 0;
    }
    N.size.assign(1, (int32_t)n_active);
  } else {
    father = N.from_father;
    N.size = fsize;
  }
  const int nc2 = (int)N.cell.size();
  if ((int)N.size.size() != nc2) return false;
  N.slot_ptr.assign(nc2 + 1, 0);
  for (int c = 0; c < nc2; ++c) N.slot_ptr[c + 1] = N.slot_ptr[c] + N.size[c];
  N.slots.assign(N.slot_ptr[nc2], 0);
  for (int p = 0; p < cs; ++p) {
    const int a = C.seps[p];
    const int r = C.post_size(a);
    std::copy(C.slots.begin() + C.slot_ptr[a], C.slots.begin() + C.slot_ptr[a] + r,
              N.slots.begin() + N.slot_ptr[father[p]] + loc[p]);
  }
  build_offsets(N, P.pi, P.opt.compression);
  N.cp_father = father;
  N.cp_loc = loc;
  if (!emit) {
    validate_level(N, P.n, P.pi);
    return true;
  }
  emit_copy_maps(C, N, father, loc, P.pi, blk_map, phi_map);
  validate_level(N, P.n, P.pi);
  validate_copies(blk_map, C.front_elems + C.blk_elems, N.front_elems + N.blk_elems);
  validate_copies(phi_map, C.phi_elems, N.phi_elems);
  return true;
}

}  // namespace sgf
