// Tiled multi-workgroup elimination for large fronts and for the top node.
//
// A level whose fronts are too large for one workgroup's LDS panel, or too
// few to fill the chip, is eliminated (Eq. 4.2) by a sequence of level-wide
// launches, all fronts of the level together:
//   for every 64-column panel p of the eliminated block:
//     k_tdiag:   factor the diagonal tile;
//     k_tpanel:  solve the rows below it (TRSM);
//     k_tupdate: subtract the panel's outer product from the remaining
//                eliminated columns (matrix cores);
//   k_tschur:   M_SS -= L_SI L_SI^T in one deep contraction (matrix cores).
// The same sweep also builds Zt = L_II^{-T}: the front is extended by m
// identity rows (A_SI := I gives L_SI = L_II^{-T}), and the rows of Zt that
// are known to be zero are skipped.  The preconditioner apply of such a
// front is then four matrix-vector products with full parallelism instead of
// a chain of triangular solves.
#pragma once

#include "sgf_kernels.hpp"

namespace sgf {

constexpr int TB = 64;       // tile edge and panel width
constexpr int TROWS = 256;   // rows per panel workgroup, one per thread
constexpr int TKC = 32;      // depth of one LDS stage of a tile contraction

struct TFront {
  int64_t f_off;      // front (R x R, column-major, ld R) in the factor buffer
  int64_t z_off;      // Zt = L_II^{-T} (m x m, column-major, ld m), upper triangular
  int64_t u_off;      // m-vector of the apply work buffer
  int64_t slot_off;   // slots of I
  int64_t nslot_off;  // slots of the neighbours (k entries)
  int64_t t_off;      // apply scratch (k entries)
  int32_t R, m, cluster;
  int32_t zrows;      // rows of Zt formed alongside: m, or 0 when not wanted
};

template <typename TS, typename TD>
__global__ void k_convert(const TS* __restrict__ src, TD* __restrict__ dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (TD)src[i];
}

// Zt <- I for every front.
template <typename T>
__global__ void k_tinit(const TFront* __restrict__ D, T* __restrict__ zb) {
  const TFront d = D[blockIdx.y];
  if (d.zrows == 0) return;
  const int64_t mm = (int64_t)d.m * d.m;
  T* Z = zb + d.z_off;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < mm; i += (int64_t)gridDim.x * blockDim.x)
    Z[i] = (i % d.m == i / d.m) ? T(1) : T(0);
}

// Panel p, diagonal tile: F[c0:c0+w, c0:c0+w] <- chol (lower), one
// workgroup per front, in wave 0's registers (lane i holds row i, pivots
// broadcast through scalar registers).  A non-positive pivot sets *fail to
// the cluster id and continues with pivot 1.
template <typename T>
__global__ __launch_bounds__(WAVE) void k_tdiag(const TFront* __restrict__ D, int p, T* __restrict__ fb,
                                                int* fail) {
  const TFront d = D[blockIdx.x];
  const int R = d.R, m = d.m, c0 = p * TB;
  if (c0 >= m) return;
  const int w = min(TB, m - c0);
  T* F = fb + d.f_off;
  const int lane = threadIdx.x;
  T a[TB];
#pragma unroll
  for (int k = 0; k < TB; ++k)
    a[k] = (lane < w && k < w && k <= lane) ? F[(c0 + lane) + (int64_t)(c0 + k) * R] : T(0);
#pragma unroll
  for (int j = 0; j < TB; ++j) {
    if (j < w) {
      T dj = lane_bcast(a[j], j);
      if (!(dj > T(0))) {
        if (lane == 0) atomicCAS(fail, -1, d.cluster);
        dj = T(1);
      }
      const T sd = sqrt(dj), inv = T(1) / sd;
      const T l = (lane == j) ? sd : a[j] * inv;
      if (lane >= j) a[j] = l;
#pragma unroll
      for (int k = j + 1; k < TB; ++k) {
        const T lk = lane_bcast(l, k);
        if (lane >= k) a[k] -= l * lk;
      }
    }
  }
  if (lane < w) {
#pragma unroll
    for (int k = 0; k < TB; ++k)
      if (k <= lane && k < w) F[(c0 + lane) + (int64_t)(c0 + k) * R] = a[k];
  }
}

// Panel p, rows below the diagonal tile: each thread solves one row,
// x <- x L_pp^{-T}, with L_pp (already factored) staged in LDS.  Rows
// 0..R-1 are front rows, rows R..R+m-1 are rows of Zt; a Zt row r' is still
// zero in this panel when r' >= c0 + w.
template <typename T>
__global__ __launch_bounds__(WG) void k_tpanel(const TFront* __restrict__ D, int p, T* __restrict__ fb,
                                               T* __restrict__ zb) {
  __shared__ T Ls[TB * TB];   // L_pp row-major
  __shared__ T rinv[TB];
  const TFront d = D[blockIdx.y];
  const int R = d.R, m = d.m, c0 = p * TB;
  if (c0 >= m) return;
  const int w = min(TB, m - c0);
  const int r_lo = blockIdx.x * TROWS;
  const int fr_lo = max(r_lo, c0 + w), fr_hi = min(r_lo + TROWS, R);
  const int er_lo = max(r_lo - R, 0), er_hi = min(min(r_lo + TROWS - R, d.zrows), c0 + w);
  if (fr_lo >= fr_hi && er_lo >= er_hi) return;
  T* F = fb + d.f_off;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < TB * TB; idx += WG) {
    const int i = idx % TB, k = idx / TB;   // column-major walk: coalesced reads
    Ls[i * TB + k] = (i < w && k <= i) ? F[(c0 + i) + (int64_t)(c0 + k) * R] : T(0);
  }
  __syncthreads();
  if (tid < w) rinv[tid] = T(1) / Ls[tid * TB + tid];
  __syncthreads();
  const int r = r_lo + tid;
  T* row = nullptr;
  int64_t ld = 0;
  if (r >= fr_lo && r < fr_hi) {
    row = F + r;
    ld = R;
  } else if (r >= R && r - R >= er_lo && r - R < er_hi) {
    row = zb + d.z_off + (r - R);
    ld = m;
  }
  if (row == nullptr) return;
  T x[TB];
#pragma unroll
  for (int k = 0; k < TB; ++k) x[k] = k < w ? row[(int64_t)(c0 + k) * ld] : T(0);
#pragma unroll
  for (int j = 0; j < TB; ++j) {
    if (j < w) {
      T acc = x[j];
#pragma unroll
      for (int q = 0; q < j; ++q) acc -= x[q] * Ls[j * TB + q];
      x[j] = acc * rinv[j];
    }
  }
#pragma unroll
  for (int k = 0; k < TB; ++k)
    if (k < w) row[(int64_t)(c0 + k) * ld] = x[k];
}

// C[i][j] -= sum_{k < kc} A[i][k] B[j][k] for one 64 x 64 tile on the matrix
// cores (i < crows, j < ccols, and i >= j when `lower`).  A[i][k] is
// A[i + k lda], B[j][k] is B[j + k ldb], C[i][j] is C[i + j ldc].  Operands are
// staged through LDS in stages of TKC columns, the next stage held in
// registers while the current one is multiplied.  Each wavefront owns a
// 32 x 32 quarter, computed as its transpose so that lane % 16 walks rows of
// the column-major C; the product is added to C once at the end.
template <typename T>
__device__ void tile_gemm_nt(const T* __restrict__ A, int64_t lda, int arows, const T* __restrict__ B,
                             int64_t ldb, int brows, int kc, T* __restrict__ C, int64_t ldc, int crows,
                             int ccols, bool lower, T* sA, T* sB) {
  typedef typename Mfma<T>::V V;
  const int tid = threadIdx.x, lane = tid % WAVE, wv = tid / WAVE;
  const int li = lane % 16, lk = lane / 16;
  const int b0 = 32 * (wv / 2), a0 = 32 * (wv % 2);   // C rows (b) and C columns (a) of this wave
  V acc[2][2];
#pragma unroll
  for (int ia = 0; ia < 2; ++ia)
#pragma unroll
    for (int ib = 0; ib < 2; ++ib)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[ia][ib][v] = T(0);
  constexpr int PER = TB * TKC / WG;   // elements of each operand per thread and stage
  constexpr int KSTEP = WG / TB;       // stage columns between a thread's elements
  const int fi = tid % TB, fk = tid / TB;
  const bool aok = fi < arows, bok = fi < brows;
  const T* pa = A + fi + (int64_t)fk * lda;
  const T* pb = B + fi + (int64_t)fk * ldb;
  T ra[PER], rb[PER];
  auto fetch = [&](int k0) {
    const T* qa = pa + (int64_t)k0 * lda;
    const T* qb = pb + (int64_t)k0 * ldb;
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const bool kin = k0 + fk + KSTEP * e < kc;
      ra[e] = (kin && aok) ? qa[(int64_t)(KSTEP * e) * lda] : T(0);
      rb[e] = (kin && bok) ? qb[(int64_t)(KSTEP * e) * ldb] : T(0);
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < kc; k0 += TKC) {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      sA[tid + e * WG] = ra[e];
      sB[tid + e * WG] = -rb[e];
    }
    __syncthreads();
    if (k0 + TKC < kc) fetch(k0 + TKC);
#pragma unroll
    for (int ks = 0; ks < TKC; ks += 4) {
      const int k = ks + lk;
      const T oa0 = sB[k * TB + a0 + li], oa1 = sB[k * TB + a0 + 16 + li];
      const T ob0 = sA[k * TB + b0 + li], ob1 = sA[k * TB + b0 + 16 + li];
      acc[0][0] = Mfma<T>::op(oa0, ob0, acc[0][0]);
      acc[0][1] = Mfma<T>::op(oa0, ob1, acc[0][1]);
      acc[1][0] = Mfma<T>::op(oa1, ob0, acc[1][0]);
      acc[1][1] = Mfma<T>::op(oa1, ob1, acc[1][1]);
    }
  }
#pragma unroll
  for (int ia = 0; ia < 2; ++ia)
#pragma unroll
    for (int ib = 0; ib < 2; ++ib) {
      const int i = b0 + 16 * ib + li;
      if (i >= crows) continue;
      T* ci = C + i;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = a0 + 16 * ia + Mfma<T>::drow(lane, v);
        if (j < ccols && (!lower || i >= j)) ci[(int64_t)j * ldc] += acc[ia][ib][v];
      }
    }
}

// After panel p: the eliminated columns [c0 + 64, m) lose the panel's outer
// product, on front rows at or below the column tile and on the Zt rows of
// tiles 0..p (the others are still zero).  Work item = (column tile jt, row
// tile rt); rt < nft are front row tiles, the rest Zt row tiles.
template <typename T>
__global__ __launch_bounds__(WG) void k_tupdate(const TFront* __restrict__ D, int p, T* __restrict__ fb,
                                                T* __restrict__ zb) {
  __shared__ T sA[TB * TKC], sB[TB * TKC];
  const TFront d = D[blockIdx.y];
  const int R = d.R, m = d.m, c0 = p * TB;
  if (c0 + TB >= m) return;
  const int nct = (m + TB - 1) / TB, nj = nct - p - 1;
  const int nft = (R + TB - 1) / TB, nrt = nft + (d.zrows > 0 ? p + 1 : 0);
  const int t = blockIdx.x;
  if (t >= nj * nrt) return;
  const int jt = p + 1 + t % nj, rt = t / nj;
  T* F = fb + d.f_off;
  const T* rowbase;
  T* cbase;
  int64_t ld;
  int nrows;
  bool lower = false;
  if (rt < nft) {
    if (rt < jt) return;
    rowbase = F + TB * rt;
    cbase = F + TB * rt;
    ld = R;
    nrows = min(TB, R - TB * rt);
    lower = rt == jt;
  } else {
    const int ie = rt - nft;
    T* Z = zb + d.z_off;
    rowbase = Z + TB * ie;
    cbase = Z + TB * ie;
    ld = m;
    nrows = min(TB, m - TB * ie);
  }
  const int col0 = TB * jt, ncols = min(TB, m - col0);
  tile_gemm_nt<T>(rowbase + (int64_t)c0 * ld, ld, nrows, F + col0 + (int64_t)c0 * R, R, ncols, TB,
                  cbase + (int64_t)col0 * ld, ld, nrows, ncols, lower, sA, sB);
}

// M_SS -= L_SI L_SI^T: one 64 x 64 tile of the lower triangle of the Schur
// block per work item, contracted over all m eliminated columns.
template <typename T>
__global__ __launch_bounds__(WG) void k_tschur(const TFront* __restrict__ D, T* __restrict__ fb) {
  __shared__ T sA[TB * TKC], sB[TB * TKC];
  const TFront d = D[blockIdx.y];
  const int R = d.R, m = d.m, k = R - m;
  const int nst = (k + TB - 1) / TB;
  const int t = blockIdx.x;
  if (t >= nst * nst) return;
  const int jt = t % nst, it = t / nst;
  if (it < jt) return;
  T* F = fb + d.f_off;
  const int r0 = m + TB * it, q0 = m + TB * jt;
  const int nrows = min(TB, R - r0), ncols = min(TB, R - q0);
  tile_gemm_nt<T>(F + r0, R, nrows, F + q0, R, ncols, m, F + r0 + (int64_t)q0 * R, R, nrows, ncols, it == jt, sA,
                  sB);
}

// ---------------------------------------------------------------------------
// Apply of tiled fronts (Sec. 4.7).  Vectors in the sweep precision TV, the
// factor and the work vector u in TF.
// ---------------------------------------------------------------------------

// u = Z y_I with Z = Zt^T (lower): u[c] = sum_{r <= c} Zt[r][c] y_I[r].  One
// wavefront per column, 64 columns per workgroup, rc right-hand sides
// (columns blockIdx.z * rc ...) sharing each factor load.
template <typename TV, typename TF>
__global__ __launch_bounds__(WG) void k_tfwd_z(const TFront* __restrict__ D, const TF* __restrict__ zb,
                                               const int32_t* __restrict__ slots, const TV* __restrict__ y,
                                               int64_t ldy, TF* __restrict__ uw, int64_t ldu, int nrhs, int rc) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  TF* ys = reinterpret_cast<TF*>(smem_raw);
  const TFront d = D[blockIdx.y];
  const int m = d.m, cb = blockIdx.x * TB;
  if (cb >= m) return;
  const int ce = min(cb + TB, m);
  const int q0 = blockIdx.z * rc, nc = min(rc, nrhs - q0);
  const int32_t* sl = slots + d.slot_off;
  for (int idx = threadIdx.x; idx < ce * nc; idx += WG) {
    const int i = idx % ce, q = idx / ce;
    ys[i + q * ce] = (TF)y[(int64_t)(q0 + q) * ldy + sl[i]];
  }
  __syncthreads();
  const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
  const TF* Z = zb + d.z_off;
  for (int c = cb + wv; c < ce; c += WG / WAVE) {
    const TF* zc = Z + (int64_t)c * m;
    TF acc[RCM];
#pragma unroll
    for (int q = 0; q < RCM; ++q) acc[q] = 0;
    for (int r = lane; r <= c; r += WAVE) {
      const TF z = zc[r];
#pragma unroll
      for (int q = 0; q < RCM; ++q)
        if (q < nc) acc[q] += z * ys[r + q * ce];
    }
#pragma unroll
    for (int q = 0; q < RCM; ++q)
      if (q < nc) {
        const TF t = wave_sum(acc[q]);
        if (lane == 0) uw[(int64_t)(q0 + q) * ldu + d.u_off + c] = t;
      }
  }
}

// t = L_SI u into the apply scratch (the separators subtract it later), and
// y_I <- u.  64 rows of L_SI per workgroup, the columns split over the four
// wavefronts and their partial sums added in a fixed order.
template <typename TV, typename TF>
__global__ __launch_bounds__(WG) void k_tfwd_s(const TFront* __restrict__ D, const TF* __restrict__ fb,
                                               const TF* __restrict__ uw, int64_t ldu,
                                               const int32_t* __restrict__ slots, TV* __restrict__ y, int64_t ldy,
                                               TV* __restrict__ tscr, int64_t ldt, int nrhs, int rc) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  TF* us = reinterpret_cast<TF*>(smem_raw);
  const TFront d = D[blockIdx.y];
  const int m = d.m, R = d.R, k = R - m, mp = (m + 3) & ~3;
  const int rb = blockIdx.x * TB;
  const int q0 = blockIdx.z * rc, nc = min(rc, nrhs - q0);
  if (blockIdx.x == 0) {
    const int32_t* sl = slots + d.slot_off;
    for (int idx = threadIdx.x; idx < m * nc; idx += WG) {
      const int i = idx % m, q = idx / m;
      y[(int64_t)(q0 + q) * ldy + sl[i]] = (TV)uw[(int64_t)(q0 + q) * ldu + d.u_off + i];
    }
  }
  if (rb >= k) return;
  for (int idx = threadIdx.x; idx < m * nc; idx += WG) {
    const int i = idx % m, q = idx / m;
    us[i + q * mp] = uw[(int64_t)(q0 + q) * ldu + d.u_off + i];
  }
  TF* part = us + mp * rc;
  __syncthreads();
  const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
  const int a = rb + lane;
  TF acc[RCM];
#pragma unroll
  for (int q = 0; q < RCM; ++q) acc[q] = 0;
  if (a < k) {
    const TF* L = fb + d.f_off + m + a;
#pragma unroll 4
    for (int c = wv; c < m; c += WG / WAVE) {
      const TF l = L[(int64_t)c * R];
#pragma unroll
      for (int q = 0; q < RCM; ++q)
        if (q < nc) acc[q] += l * us[c + q * mp];
    }
  }
#pragma unroll
  for (int q = 0; q < RCM; ++q)
    if (q < nc) part[(q * (WG / WAVE) + wv) * WAVE + lane] = acc[q];
  __syncthreads();
  if (wv < nc && a < k) {
    const TF* pq = part + wv * (WG / WAVE) * WAVE;
    TF sum = pq[lane];
    for (int w = 1; w < WG / WAVE; ++w) sum += pq[w * WAVE + lane];
    tscr[(int64_t)(q0 + wv) * ldt + d.t_off + a] = (TV)sum;
  }
}

// v = y_I - L_SI^T y_S: one wavefront per column of L_SI.
template <typename TV, typename TF>
__global__ __launch_bounds__(WG) void k_tbwd_s(const TFront* __restrict__ D, const TF* __restrict__ fb,
                                               const int32_t* __restrict__ slots,
                                               const int32_t* __restrict__ nslots, const TV* __restrict__ y,
                                               int64_t ldy, TF* __restrict__ uw, int64_t ldu, int nrhs, int rc) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  TF* ysS = reinterpret_cast<TF*>(smem_raw);
  const TFront d = D[blockIdx.y];
  const int m = d.m, R = d.R, k = R - m, cb = blockIdx.x * TB;
  if (cb >= m) return;
  const int ce = min(cb + TB, m);
  const int q0 = blockIdx.z * rc, nc = min(rc, nrhs - q0);
  const int32_t* ns = nslots + d.nslot_off;
  for (int idx = threadIdx.x; idx < k * nc; idx += WG) {
    const int i = idx % k, q = idx / k;
    ysS[i + q * k] = (TF)y[(int64_t)(q0 + q) * ldy + ns[i]];
  }
  __syncthreads();
  const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
  const int32_t* sl = slots + d.slot_off;
  for (int c = cb + wv; c < ce; c += WG / WAVE) {
    const TF* lc = fb + d.f_off + m + (int64_t)c * R;
    TF acc[RCM];
#pragma unroll
    for (int q = 0; q < RCM; ++q) acc[q] = 0;
    for (int a = lane; a < k; a += WAVE) {
      const TF l = lc[a];
#pragma unroll
      for (int q = 0; q < RCM; ++q)
        if (q < nc) acc[q] += l * ysS[a + q * k];
    }
#pragma unroll
    for (int q = 0; q < RCM; ++q)
      if (q < nc) {
        const TF t = wave_sum(acc[q]);
        if (lane == 0)
          uw[(int64_t)(q0 + q) * ldu + d.u_off + c] = (TF)y[(int64_t)(q0 + q) * ldy + sl[c]] - t;
      }
  }
}

// y_I = Zt v (upper): y_I[r] = sum_{c >= r} Zt[r][c] v[c].  64 rows per
// workgroup, columns split over the wavefronts, fixed-order partial sums.
template <typename TV, typename TF>
__global__ __launch_bounds__(WG) void k_tbwd_z(const TFront* __restrict__ D, const TF* __restrict__ zb,
                                               const TF* __restrict__ uw, int64_t ldu,
                                               const int32_t* __restrict__ slots, TV* __restrict__ y, int64_t ldy,
                                               int nrhs, int rc) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  TF* vs = reinterpret_cast<TF*>(smem_raw);
  const TFront d = D[blockIdx.y];
  const int m = d.m, rb = blockIdx.x * TB;
  if (rb >= m) return;
  const int q0 = blockIdx.z * rc, nc = min(rc, nrhs - q0);
  const int len = m - rb, lp = (len + 3) & ~3;
  for (int idx = threadIdx.x; idx < len * nc; idx += WG) {
    const int i = idx % len, q = idx / len;
    vs[i + q * lp] = uw[(int64_t)(q0 + q) * ldu + d.u_off + rb + i];
  }
  TF* part = vs + lp * rc;
  __syncthreads();
  const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
  const int r = rb + lane;
  TF acc[RCM];
#pragma unroll
  for (int q = 0; q < RCM; ++q) acc[q] = 0;
  if (r < m) {
    const TF* zr = zb + d.z_off + r;
#pragma unroll 4
    for (int c = rb + wv; c < m; c += WG / WAVE)
      if (c >= r) {
        const TF z = zr[(int64_t)c * m];
#pragma unroll
        for (int q = 0; q < RCM; ++q)
          if (q < nc) acc[q] += z * vs[c - rb + q * lp];
      }
  }
#pragma unroll
  for (int q = 0; q < RCM; ++q)
    if (q < nc) part[(q * (WG / WAVE) + wv) * WAVE + lane] = acc[q];
  __syncthreads();
  if (wv < nc && r < m) {
    const TF* pq = part + wv * (WG / WAVE) * WAVE;
    TF sum = pq[lane];
    for (int w = 1; w < WG / WAVE; ++w) sum += pq[w * WAVE + lane];
    y[(int64_t)(q0 + wv) * ldy + slots[d.slot_off + r]] = (TV)sum;
  }
}

}  // namespace sgf
