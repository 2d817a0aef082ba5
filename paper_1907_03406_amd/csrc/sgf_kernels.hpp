// Device kernels of the SGF factorization, apply and CG for gfx950.
//
// All kernels are batched over the clusters of one tree level: one
// workgroup of 256 threads (four 64-wide wavefronts) per cluster, clusters
// of uneven sizes described by the planner's descriptor tables.  Every sum
// whose terms come from different clusters is formed by a gather in a fixed
// order (no floating-point atomics), so results are deterministic.
#pragma once

#include <hip/hip_runtime.h>

#include "sgf_plan.hpp"

namespace sgf {

constexpr int WG = 256;
constexpr int WAVE = 64;
constexpr double TIE_RTOL = 1e-10;

// Nearest bfloat16 (ties to even) of an FP32 value, as FP32; FP64 values
// pass through the FP32 rounding first.
__device__ __forceinline__ float bf16_round(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}
__device__ __forceinline__ double bf16_round(double x) { return (double)bf16_round((float)x); }
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

// Value of v in lane `src` (a wave-uniform index) for every lane, through a
// scalar register (v_readlane).
__device__ __forceinline__ float lane_bcast(float v, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
__device__ __forceinline__ double lane_bcast(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}

// Global memory through a buffer resource covering [base, base + bytes): an
// access at a byte offset past the end is dropped by the hardware (a load
// returns 0), so a lane with nothing to load or store passes BUF_OOB instead
// of branching around the access.  Straight-line accesses let the compiler
// count outstanding memory operations exactly, so that waiting for a load
// does not also wait for every store issued before it.
constexpr int BUF_OOB = 0x7fffffff;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_res(const void* base, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ int buf_off(bool valid, int64_t elem, int esz) {
  return valid ? (int)(elem * esz) : BUF_OOB;
}
__device__ __forceinline__ float buf_ld(__amdgpu_buffer_rsrc_t r, int off, float) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ double buf_ld(__amdgpu_buffer_rsrc_t r, int off, double) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, int off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, off, 0, 0);
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, int off, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 0);
}

// Sum over the workgroup; every thread gets the result.  `red` holds WG/WAVE.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  T s = 0;
  for (int i = 0; i < WG / WAVE; ++i) s += red[i];
  return s;
}

// 16 x 16 x 4 matrix-core step (v_mfma_*_16x16x4).  Operand lane layout,
// checked on gfx950: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16];
// the result D[i][j] sits in lane j + 16 (i / 4), register i % 4 (f32) or in
// lane j + 16 (i % 4), register i / 4 (f64).  `drow` gives, for a lane and a
// register, the row index i of D that it holds.
typedef float mfma_v4f __attribute__((ext_vector_type(4)));
typedef double mfma_v4d __attribute__((ext_vector_type(4)));
template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
  typedef mfma_v4f V;
  static __device__ __forceinline__ V op(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int drow(int lane, int v) { return 4 * (lane / 16) + v; }
};
template <>
struct Mfma<double> {
  typedef mfma_v4d V;
  static __device__ __forceinline__ V op(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int drow(int lane, int v) { return lane / 16 + 4 * v; }
};

// The bfloat16 bits of that nearest value.
__device__ __forceinline__ short bf16_bits(float x) { return (short)(__float_as_uint(bf16_round(x)) >> 16); }

// 16 x 16 x 16 bfloat16 matrix-core step with FP32 accumulation
// (v_mfma_f32_16x16x16_bf16).  Operand lane layout, checked on gfx950: lane l
// supplies A[l % 16][4 (l / 16) + e] and B[4 (l / 16) + e][l % 16], e = 0..3;
// D[4 (l / 16) + v][l % 16] sits in lane l, register v.
typedef short mfma_v4bf __attribute__((ext_vector_type(4)));
__device__ __forceinline__ mfma_v4f mfma_bf16(mfma_v4bf a, mfma_v4bf b, mfma_v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// One wavefront forms rows i0 .. i0 + 15 of D (rows x cols, cols <= 16,
// ld ldd) = A B from operands rounded to bfloat16, on the matrix cores: A is
// rows x kk, read as a(i, j); B is kk x cols, read as b(j, p); entries
// outside the extents are zero.
template <typename T, typename FA, typename FB>
__device__ __forceinline__ void wave_bf16_tile(int i0, int rows, int cols, int kk, FA a, FB b, T* D, int64_t ldd) {
  const int lane = threadIdx.x % WAVE, r16 = lane % 16, k4 = 4 * (lane / 16);
  mfma_v4f acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < kk; k0 += 16) {
    mfma_v4bf av, bv;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int ia = i0 + r16, ja = k0 + k4 + e;
      av[e] = (ia < rows && ja < kk) ? bf16_bits((float)a(ia, ja)) : (short)0;
      bv[e] = (ja < kk && r16 < cols) ? bf16_bits((float)b(ja, r16)) : (short)0;
    }
    acc = mfma_bf16(av, bv, acc);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = i0 + k4 + v;
    if (i < rows && r16 < cols) D[i + (int64_t)r16 * ldd] = (T)acc[v];
  }
}
// All row tiles by one wavefront.
template <typename T, typename FA, typename FB>
__device__ __forceinline__ void wave_bf16_gemm(int rows, int cols, int kk, FA a, FB b, T* D, int64_t ldd) {
  for (int i0 = 0; i0 < rows; i0 += 16) wave_bf16_tile<T>(i0, rows, cols, kk, a, b, D, ldd);
}

// ---------------------------------------------------------------------------
// Fills and copies
// ---------------------------------------------------------------------------

template <typename T>
__global__ void k_fill_csr(const double* __restrict__ vals, const int64_t* __restrict__ dst,
                           int64_t nnz, T* __restrict__ arena) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nnz) {
    int64_t d = dst[e];
    if (d >= 0) arena[d] = (T)vals[e];
  }
}

template <typename T>
__global__ void k_copy_blocks(const CopyDesc* __restrict__ D, const T* __restrict__ src,
                              T* __restrict__ dst) {
  const CopyDesc d = D[blockIdx.x];
  const int64_t tot = (int64_t)d.rows * d.cols;
  for (int64_t idx = threadIdx.x; idx < tot; idx += blockDim.x) {
    int i = (int)(idx % d.rows), j = (int)(idx / d.rows);
    T v = src[d.src_off + i + (int64_t)j * d.src_ld];
    if (d.mode == 0) dst[d.dst_off + i + (int64_t)j * d.dst_ld] = v;
    else dst[d.dst_off + j + (int64_t)i * d.dst_ld] = v;
  }
}

// Two copy maps in one launch: workgroups [0, n1) copy by D1 from src1 to
// dst1, the rest by D2 from src2 to dst2 (each as k_copy_blocks).
template <typename T>
__global__ void k_copy_blocks2(const CopyDesc* __restrict__ D1, const T* __restrict__ src1, T* __restrict__ dst1,
                               int n1, const CopyDesc* __restrict__ D2, const T* __restrict__ src2,
                               T* __restrict__ dst2) {
  const bool first = (int)blockIdx.x < n1;
  const CopyDesc d = first ? D1[blockIdx.x] : D2[blockIdx.x - n1];
  const T* src = first ? src1 : src2;
  T* dst = first ? dst1 : dst2;
  const int64_t tot = (int64_t)d.rows * d.cols;
  for (int64_t idx = threadIdx.x; idx < tot; idx += blockDim.x) {
    int i = (int)(idx % d.rows), j = (int)(idx / d.rows);
    T v = src[d.src_off + i + (int64_t)j * d.src_ld];
    if (d.mode == 0) dst[d.dst_off + i + (int64_t)j * d.dst_ld] = v;
    else dst[d.dst_off + j + (int64_t)i * d.dst_ld] = v;
  }
}

// Coarsening (Secs. 4.3-4.4, Eq. 4.7) with the destinations computed here:
// item q < np copies the coarse part (ra x rb, ra / rb the sizes after the
// compressions) of pair block q of the level below into the new level's
// arena, at the place its CoarsenPair kind says (the kinds of the host copy
// maps), with its transpose where the block lands in a symmetric
// position; item np + p copies the Phi rows of separator p into its
// father's Phi.  Every table index and every source and destination range
// is checked against its table or buffer first; one outside sets *err and
// the item copies nothing.
template <typename T>
__global__ __launch_bounds__(WG) void k_coarsen(
    const PairDesc* __restrict__ CP, const CoarsenPair* __restrict__ map, int np, const CoarsenSep* __restrict__ seps,
    int ns, const int* __restrict__ rank, const int32_t* __restrict__ father, const int32_t* __restrict__ loc,
    const ElimDesc* __restrict__ NE, int n_ne, const PairDesc* __restrict__ NP, int n_np,
    const int32_t* __restrict__ nbr_off, int64_t n_nbr, int n_clusters, int n_comp, const T* __restrict__ carena, int64_t c_front, int64_t c_elems, T* __restrict__ narena, int64_t n_front,
    int64_t n_elems, const int64_t* __restrict__ c_slotptr, const int64_t* __restrict__ c_phioff,
    const T* __restrict__ cphi, int64_t c_phi_elems, const int64_t* __restrict__ n_slotptr,
    const int64_t* __restrict__ n_phioff, T* __restrict__ nphi, int64_t n_phi_elems, int pi, int do_phi,
    int* __restrict__ err) {
  const int item = blockIdx.x;
  if (item < np) {
    const PairDesc pd = CP[item];
    const CoarsenPair mp = map[item];
    const bool idx_ok = pd.ca < n_comp && pd.cb < n_comp && mp.pa >= 0 && mp.pa < ns && mp.pb >= 0 && mp.pb < ns &&
                        mp.tgt >= 0 && ((mp.kind <= 0 || mp.kind > 5) ? mp.kind == 0 && mp.tgt < n_ne
                                        : mp.kind == 1 || mp.kind >= 4 ? mp.tgt < n_np
                                        : mp.tgt < n_ne && mp.e >= 0 && mp.e < n_nbr);
    if (!idx_ok) {
      if (threadIdx.x == 0) atomicExch(err, 1);
      return;
    }
    const int ra = (pd.ca >= 0 && rank[pd.ca] < pd.s_a) ? rank[pd.ca] : pd.s_a;
    const int rb = (pd.cb >= 0 && rank[pd.cb] < pd.s_b) ? rank[pd.cb] : pd.s_b;
    if (ra == 0 || rb == 0) return;
    const int oa = loc[mp.pa], ob = loc[mp.pb];
    const int64_t src = c_front + pd.blk_off, sld = pd.s_a;
    // destination of the block (d0) and of its transpose (d1)
    const CoarsenDst cd = coarsen_dest(mp.kind, mp.tgt, mp.e, oa, ob, pd.a == pd.b, NE, NP, nbr_off, n_front);
    const int64_t d0 = cd.d0, d1 = cd.d1, ld = cd.ld;
    bool ok = mp.kind >= 0 && mp.kind <= 5 && src >= 0 && src + (ra - 1) + (int64_t)(rb - 1) * sld < c_elems;
    if (d0 >= 0) ok = ok && d0 + (ra - 1) + (int64_t)(rb - 1) * ld < n_elems;
    if (d1 >= 0) ok = ok && d1 + (rb - 1) + (int64_t)(ra - 1) * ld < n_elems;
    if (d0 < 0 && d1 < 0) ok = false;
    if (!ok) {
      if (threadIdx.x == 0) atomicExch(err, 1);
      return;
    }
    for (int idx = threadIdx.x; idx < ra * rb; idx += WG) {
      const int i = idx % ra, j = idx / ra;
      const T v = carena[src + i + (int64_t)j * sld];
      if (d0 >= 0) narena[d0 + i + (int64_t)j * ld] = v;
      if (d1 >= 0) narena[d1 + j + (int64_t)i * ld] = v;
    }
    return;
  }
  const int p = item - np;
  if (!do_phi || p >= ns) return;
  const CoarsenSep cs = seps[p];
  if (cs.cluster < 0 || cs.ci >= n_comp || father[p] < 0 || father[p] >= n_clusters) {
    if (threadIdx.x == 0) atomicExch(err, 1);
    return;
  }
  const int sa = (int)(c_slotptr[cs.cluster + 1] - c_slotptr[cs.cluster]);
  const int r = (cs.ci >= 0 && rank[cs.ci] < sa) ? rank[cs.ci] : sa;
  if (r == 0) return;
  const int D = father[p];
  const int64_t dld = n_slotptr[D + 1] - n_slotptr[D];
  const int64_t s0 = c_phioff[cs.cluster], d0 = n_phioff[D] + loc[p];
  const bool ok = s0 >= 0 && d0 >= 0 && s0 + (r - 1) + (int64_t)(pi - 1) * sa < c_phi_elems &&
                  d0 + (r - 1) + (int64_t)(pi - 1) * dld < n_phi_elems && loc[p] + r <= dld;
  if (!ok) {
    if (threadIdx.x == 0) atomicExch(err, 1);
    return;
  }
  for (int idx = threadIdx.x; idx < r * pi; idx += WG) {
    const int i = idx % r, j = idx / r;
    nphi[d0 + i + (int64_t)j * dld] = cphi[s0 + i + (int64_t)j * sa];
  }
}

template <typename T>
__global__ void k_zero(T* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = T(0);
}

// Several descriptor tables uploaded as one blob: a header of pieces (offset
// of the table in the blob, its device destination, its size in bytes, a
// multiple of 4) followed by the tables.  Workgroup (p, c) copies chunk c of
// piece p.
struct BlobPiece {
  uint64_t src_off, dst, bytes;
};
constexpr int BLOB_CHUNK = WG * 16;   // 4-byte words per workgroup
__global__ __launch_bounds__(WG) void k_scatter_blob(const unsigned char* __restrict__ blob) {
  const BlobPiece pc = reinterpret_cast<const BlobPiece*>(blob)[blockIdx.x];
  const int64_t words = (int64_t)(pc.bytes / 4);
  const int64_t lo = (int64_t)blockIdx.y * BLOB_CHUNK;
  if (lo >= words) return;
  const int64_t hi = min(words, lo + (int64_t)BLOB_CHUNK);
  const uint32_t* __restrict__ src = reinterpret_cast<const uint32_t*>(blob + pc.src_off);
  uint32_t* __restrict__ dst = reinterpret_cast<uint32_t*>(pc.dst);
  for (int64_t i = lo + threadIdx.x; i < hi; i += WG) dst[i] = src[i];
}

// Clear the entries of the fronts in `list` that the banded elimination
// reads: the lower band of M_II (rows c .. c + bw of column c, bw clamped to
// m - 1) and M_SI (rows m .. m + k - 1 of every interior column).  Valid only
// while the rest of each front is known to hold zeros, apart from the upper
// band (rewritten by the CSR fill) and the lower triangle of the separator
// block (overwritten by the banded elimination).  One workgroup per front.
template <typename T>
__global__ __launch_bounds__(WG) void k_zero_band(const ElimDesc* __restrict__ D, const int32_t* __restrict__ list,
                                                  T* __restrict__ arena) {
  const ElimDesc d = D[list[blockIdx.x]];
  const int m = d.m, k = d.k, bw = min(d.bw, max(m - 1, 0));
  const int64_t R = (int64_t)m + k;
  T* C = arena + d.front_off;
  const int lane = threadIdx.x % WAVE;
  // one column per wavefront at a time: its band segment, then its M_SI rows
  for (int c = threadIdx.x / WAVE; c < m; c += WG / WAVE) {
    T* col = C + (int64_t)c * R;
    const int nb = min(bw, m - 1 - c) + 1;
    for (int r = lane; r < nb; r += WAVE) col[c + r] = T(0);
    for (int r = lane; r < k; r += WAVE) col[m + r] = T(0);
  }
}

// Level-1 inputs of one banded front per workgroup: the band and the M_SI
// rows (all that the banded elimination reads, as k_zero_band clears them)
// set to zero with every lane busy, then, after the barrier, the front's own
// matrix entries (FP64, rounded to T) from its list, whose writes meet the
// fresh lines in L2 instead of scattering partial lines to HBM.
template <typename T>
__global__ __launch_bounds__(WG) void k_fill_band(const ElimDesc* __restrict__ D, const int32_t* __restrict__ list,
                                                  const int64_t* __restrict__ ptr, const int32_t* __restrict__ off,
                                                  const int64_t* __restrict__ src, const double* __restrict__ vals,
                                                  T* __restrict__ arena) {
  const ElimDesc d = D[list[blockIdx.x]];
  const int m = d.m, k = d.k, bw = min(d.bw, max(m - 1, 0));
  const int64_t R = (int64_t)m + k;
  T* C = arena + d.front_off;
  // the first PF entries of each thread are fetched before the clearing, so
  // that their loads overlap its stores (clamped indices: no branches)
  constexpr int PF = 8;
  const int64_t q0 = ptr[blockIdx.x], q1 = ptr[blockIdx.x + 1];
  int po[PF];
  T pv[PF];
  if (q1 > q0) {
    int64_t ps[PF];
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int64_t q = min(q0 + threadIdx.x + (int64_t)u * WG, q1 - 1);
      po[u] = off[q];
      ps[u] = src[q];
    }
#pragma unroll
    for (int u = 0; u < PF; ++u) pv[u] = (T)vals[ps[u]];
  }
  const int w2 = bw + 1 + k;   // per column: rows c .. c + bw of the band, then the k rows of M_SI
  const int n = m * w2;
  for (int e = threadIdx.x; e < n; e += WG) {
    const int c = e / w2, r = e - c * w2;
    const int row = r <= bw ? c + r : m + (r - bw - 1);
    if (r > bw || row < m) C[row + (int64_t)c * R] = T(0);
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PF; ++u)
    if (q0 + threadIdx.x + (int64_t)u * WG < q1) C[po[u]] = pv[u];
  for (int64_t q = q0 + threadIdx.x + (int64_t)PF * WG; q < q1; q += WG) C[off[q]] = (T)vals[src[q]];
}

// The level-1 entries outside the banded fronts (pair blocks).
// (four entries per thread, every load issued before the stores)
template <typename T>
__global__ void k_fill_rest(const double* __restrict__ vals, const int64_t* __restrict__ dst,
                            const int64_t* __restrict__ src, int64_t n, T* __restrict__ arena) {
  constexpr int U = 4;
  const int64_t e0 = (int64_t)blockIdx.x * blockDim.x * U + threadIdx.x;
  int64_t dd[U], ss[U];
  T vv[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t e = min(e0 + (int64_t)u * blockDim.x, n - 1);
    dd[u] = dst[e];
    ss[u] = src[e];
  }
#pragma unroll
  for (int u = 0; u < U; ++u) vv[u] = (T)vals[ss[u]];
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (e0 + (int64_t)u * blockDim.x < n) arena[dd[u]] = vv[u];
}

// Phi_B = Pi(B, :) for every level-1 cluster (Sec. 3.1; block diagonal per
// component for dofs_per_node > 1, Eq. 7.4).  Coordinates normalised
// globally to [-1, 1]: xh = (x - lo) * sc - 1 with sc = 2 / (hi - lo).
struct PhiInit {
  double lo[3], sc[3];
  int dim, q, dpn, pi, p0;
};

template <typename T>
__global__ void k_phi_init(const int64_t* __restrict__ slot_ptr, const int64_t* __restrict__ phi_off,
                           const int64_t* __restrict__ perm, const double* __restrict__ coords,
                           PhiInit pin, T* __restrict__ phi) {
  const int c = blockIdx.x;
  const int64_t s0 = slot_ptr[c];
  const int s = (int)(slot_ptr[c + 1] - s0);
  T* out = phi + phi_off[c];
  for (int i = threadIdx.x; i < s; i += blockDim.x) {
    int64_t dof = perm[s0 + i];
    int64_t node = dof / pin.dpn;
    int comp = (int)(dof % pin.dpn);
    double x[3] = {0, 0, 0};
    for (int a = 0; pin.q >= 1 && a < pin.dim; ++a) {   // q = 0 reads no coordinates
      double v = coords[node * pin.dim + a];
      x[a] = pin.sc[a] > 0 ? (v - pin.lo[a]) * pin.sc[a] - 1.0 : 0.0;
    }
    double mono[10];
    int n = 0;
    mono[n++] = 1.0;
    if (pin.q >= 1)
      for (int a = 0; a < pin.dim; ++a) mono[n++] = x[a];
    if (pin.q >= 2) {
      for (int a = 0; a < pin.dim; ++a) mono[n++] = x[a] * x[a];
      if (pin.dim == 2) mono[n++] = x[0] * x[1];
      else {
        mono[n++] = x[0] * x[1];
        mono[n++] = x[1] * x[2];
        mono[n++] = x[2] * x[0];
      }
    }
    for (int p = 0; p < pin.pi; ++p) {
      int cc = p / pin.p0, j = p % pin.p0;
      out[i + (int64_t)p * s] = (cc == comp) ? (T)mono[j] : T(0);
    }
  }
}

// Phi_B = Pi(B, :) for a basis Pi given by the user (n x pi, column major,
// FP64): any near-kernel basis in place of the monomials (Sec. 3.1).
template <typename T>
__global__ void k_phi_user(const int64_t* __restrict__ slot_ptr, const int64_t* __restrict__ phi_off,
                           const int64_t* __restrict__ perm, const double* __restrict__ basis, int64_t n, int pi,
                           T* __restrict__ phi) {
  const int c = blockIdx.x;
  const int64_t s0 = slot_ptr[c];
  const int s = (int)(slot_ptr[c + 1] - s0);
  T* out = phi + phi_off[c];
  for (int idx = threadIdx.x; idx < s * pi; idx += blockDim.x) {
    const int i = idx % s, p = idx / s;
    out[i + (int64_t)p * s] = (T)basis[perm[s0 + i] + (int64_t)p * n];
  }
}

// ---------------------------------------------------------------------------
// Workgroup dense kernels (column-major matrices in global memory)
// ---------------------------------------------------------------------------

// Partial Cholesky of the R x R front C (ld): factor the first m columns into
// [L ; L21] and subtract L21 L21^T from the trailing columns [m, nupd).
// Right-looking over panels of NB columns staged in LDS (ld padded to 4):
//  - the NB x NB diagonal block is factored by wave 0, one row per lane held
//    in registers, pivots broadcast with shuffles (no workgroup barrier);
//  - every row below it is solved against L11 by one thread (L11 read from
//    LDS as broadcasts; rows are independent);
//  - the trailing matrix is updated from the LDS panel with 4 x 4 register
//    tiles.  Three workgroup barriers per panel.
// A non-positive pivot sets *fail = code and continues with pivot 1.
// bw: lower bandwidth of the eliminated block C[0:m, 0:m] (m when dense).
// The factor keeps that band, so in panel jb the rows [jb+nb+bw, m) are
// zero: they are neither loaded, solved, written nor used in the update.
template <typename T, int NB, bool DIAG_IN_REGS>
__device__ void wg_potrf(T* __restrict__ C, int64_t ld, int R, int m, int nupd, T* lds, int* fail, int code,
                         int bw) {
  const int tid = threadIdx.x, lane = tid % WAVE, w = tid / WAVE;
  T* invd = lds;          // NB reciprocal pivots
  T* pan = lds + NB;      // panel, column p at pan + p * pl
  for (int jb = 0; jb < m; jb += NB) {
    const int nb = min(NB, m - jb);
    const int pr = R - jb;
    const int pl = (pr + 3) & ~3;
    // panel rows (local) [z0, z1) are zero; the live rows are [0, z0) and [z1, pr)
    const int z0 = min(m, jb + nb + bw) - jb, z1 = m - jb;
    const int live = z0 + (pr - z1);
    {
      // U loads in flight per thread (clamped indices), then their stores
      constexpr int U = 8;
      const int n = live * nb;
      for (int b = 0; b < n; b += U * WG) {
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int q = min(b + u * WG + tid, n - 1);
          const int ii = q % live, p = q / live;
          const int i = ii < z0 ? ii : ii - z0 + z1;
          v[u] = C[(jb + i) + (int64_t)(jb + p) * ld];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int idx = b + u * WG + tid;
          if (idx < n) {
            const int ii = idx % live, p = idx / live;
            const int i = ii < z0 ? ii : ii - z0 + z1;
            pan[p * pl + i] = v[u];
          }
        }
      }
    }
    __syncthreads();
    if (w == 0 && DIAG_IN_REGS) {
      // Cholesky of the nb x nb diagonal block: lane i keeps row i in
      // registers; column j of L is broadcast with shuffles (independent
      // across k, so they pipeline).
      T a[NB];
#pragma unroll
      for (int k = 0; k < NB; ++k) a[k] = (lane < nb && k < nb && k <= lane) ? pan[k * pl + lane] : T(0);
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        if (j < nb) {
          T d = lane_bcast(a[j], j);
          if (!(d > T(0))) {
            if (lane == 0) atomicCAS(fail, -1, code);
            d = T(1);
          }
          const T sd = sqrt(d), inv = T(1) / sd;
          const T l = (lane == j) ? sd : a[j] * inv;
          if (lane >= j) a[j] = l;
          if (lane == j) invd[j] = inv;
#pragma unroll
          for (int k = j + 1; k < NB; ++k) {
            const T lk = lane_bcast(l, k);
            if (lane >= k) a[k] -= l * lk;
          }
        }
      }
      if (lane < nb) {
#pragma unroll
        for (int k = 0; k < NB; ++k)
          if (k < nb && k <= lane) pan[k * pl + lane] = a[k];
      }
    }
    if (w == 0 && !DIAG_IN_REGS) {
      // Cholesky of the nb x nb diagonal block in LDS, right-looking, lane i
      // owns row i.  One wavefront: its LDS operations complete in program
      // order; the wave barriers only keep the compiler from moving them.
      for (int j = 0; j < nb; ++j) {
        T d = pan[j * pl + j];
        if (!(d > T(0))) {
          if (lane == 0) atomicCAS(fail, -1, code);
          d = T(1);
        }
        const T sd = sqrt(d), inv = T(1) / sd;
        __builtin_amdgcn_wave_barrier();
        if (lane == j) {
          pan[j * pl + j] = sd;
          invd[j] = inv;
        } else if (lane > j && lane < nb) {
          pan[j * pl + lane] *= inv;
        }
        __builtin_amdgcn_wave_barrier();
        if (lane > j && lane < nb) {
          const T l = pan[j * pl + lane];
          for (int k = j + 1; k <= lane; ++k) pan[k * pl + lane] -= l * pan[j * pl + k];
        }
        __builtin_amdgcn_wave_barrier();
      }
    }
    __syncthreads();
    // rows below the diagonal block: row i <- row i * L11^{-T}, one row per thread
    for (int ii = nb + tid; ii < live; ii += WG) {
      const int i = ii < z0 ? ii : ii - z0 + z1;
      for (int j = 0; j < nb; ++j) {
        T acc = pan[j * pl + i];
#pragma unroll 4
        for (int p = 0; p < j; ++p) acc -= pan[p * pl + i] * pan[p * pl + j];
        pan[j * pl + i] = acc * invd[j];
      }
    }
    __syncthreads();
    for (int idx = tid; idx < live * nb; idx += WG) {
      const int ii = idx % live, p = idx / live;
      const int i = ii < z0 ? ii : ii - z0 + z1;
      if (i >= p) C[(jb + i) + (int64_t)(jb + p) * ld] = pan[p * pl + i];
    }
    // trailing update C[i][l] -= sum_p L[i][p] L[l][p] on the matrix cores:
    // one 16 x 16 tile per wavefront step, computed as its transpose so that
    // lane % 16 walks rows (contiguous in the column-major front); the tile of
    // C is loaded into the accumulator first and -L[l][p] is fed as operand.
    const int r0 = jb + nb;
    if (r0 < nupd) {
      typedef typename Mfma<T>::V V;
      const int RT = (R - r0 + 15) / 16, CT = (nupd - r0 + 15) / 16;
      const int li = lane % 16, lk = lane / 16;
      const int zg0 = jb + z0, zg1 = jb + z1;   // zero rows / columns, global indices
      for (int t = w; t < RT * CT; t += WG / WAVE) {
        const int rt = t % RT, ct = t / RT;
        if (rt < ct) continue;
        const int i0 = r0 + 16 * rt, l0 = r0 + 16 * ct;
        if ((i0 >= zg0 && i0 + 16 <= zg1) || (l0 >= zg0 && l0 + 16 <= zg1)) continue;
        const int row = i0 + li;
        V acc;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int col = l0 + Mfma<T>::drow(lane, v);
          acc[v] = (row < R && col < nupd && row >= col) ? C[row + (int64_t)col * ld] : T(0);
        }
        const int arow = l0 + li;            // operand A': rows of the output columns
        const bool aok = arow < nupd && !(arow >= zg0 && arow < zg1);
        const bool bok = row < R && !(row >= zg0 && row < zg1);
        for (int kb = 0; kb < nb; kb += 4) {
          const int p = kb + lk;
          const T a = (aok && p < nb) ? -pan[p * pl + (arow - jb)] : T(0);
          const T b = (bok && p < nb) ? pan[p * pl + (row - jb)] : T(0);
          acc = Mfma<T>::op(a, b, acc);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int col = l0 + Mfma<T>::drow(lane, v);
          if (row < R && col < nupd && row >= col) C[row + (int64_t)col * ld] = acc[v];
        }
      }
    }
    __syncthreads();
  }
}

// LDS elements wg_potrf<T, NB> needs for a front of R rows.
__host__ __device__ inline int64_t potrf_lds_elems(int R, int nb) { return nb + (int64_t)nb * ((R + 3) & ~3); }

// X (n x ncols, ldx) <- L^{-1} X with L lower (n x n, ldl).
template <typename T>
__device__ void wg_trsm_lower(const T* __restrict__ L, int64_t ldl, int n, T* __restrict__ X,
                              int64_t ldx, int ncols) {
  for (int j = 0; j < n; ++j) {
    const T inv = T(1) / L[j + (int64_t)j * ldl];
    for (int c = threadIdx.x; c < ncols; c += WG) X[j + (int64_t)c * ldx] *= inv;
    __syncthreads();
    const int rows = n - j - 1;
    for (int idx = threadIdx.x; idx < rows * ncols; idx += WG) {
      int i = j + 1 + idx % rows, c = idx / rows;
      X[i + (int64_t)c * ldx] -= L[i + (int64_t)j * ldl] * X[j + (int64_t)c * ldx];
    }
    __syncthreads();
  }
}

// X (n x ncols, ldx) <- Q^T X, Q = H_0 ... H_{r-1}, reflector k in column k
// of V (unit diagonal implied, entries below it), coefficients tau.
template <typename T>
__device__ void wg_apply_qt(const T* __restrict__ V, int64_t ldv, const T* __restrict__ tau, int n,
                            int r, T* __restrict__ X, int64_t ldx, int ncols) {
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  for (int k = 0; k < r; ++k) {
    const T tk = tau[k];
    if (tk != T(0)) {
      for (int c = w; c < ncols; c += WG / WAVE) {
        T* x = X + (int64_t)c * ldx;
        T s = 0;
        for (int i = k + lane; i < n; i += WAVE) s += (i == k ? T(1) : V[i + (int64_t)k * ldv]) * x[i];
        s = wave_sum(s) * tk;
        for (int i = k + lane; i < n; i += WAVE) x[i] -= s * (i == k ? T(1) : V[i + (int64_t)k * ldv]);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Factorization kernels
// ---------------------------------------------------------------------------

// Work lists of the per-level launches.  With a counter (zeroed before the
// launch) the launch is persistent: a workgroup takes items from the counter
// until it passes n, the items in the order of `order` (costliest first), so
// clusters of uneven sizes balance over the resident workgroups.  Without one,
// workgroup b takes item b only.  Every workgroup leaves when the list is done.
template <bool PERS>
__device__ __forceinline__ int next_item(int* ctr, int* sh, int round, int n) {
  if constexpr (!PERS) {
    return round == 0 ? (int)blockIdx.x : n;
  } else {
    if (threadIdx.x == 0) *sh = atomicAdd(ctr, 1);
    __syncthreads();
    const int i = *sh;
    __syncthreads();
    return i;
  }
}

// Eliminate the interiors of a level (Eq. 4.2): one front at a time per
// workgroup, persistent over the level's work list.
template <typename T, int NB, bool PERS>
__global__ __launch_bounds__(WG) void k_elim(const ElimDesc* __restrict__ D, T* __restrict__ arena, int* fail,
                                             const int32_t* __restrict__ order, int n, int* ctr) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int sh;
  T* lds = reinterpret_cast<T*>(smem_raw);
  for (int round = 0; PERS || round == 0; ++round) {
    const int it = next_item<PERS>(ctr, &sh, round, n);
    if (it >= n) break;
    const ElimDesc d = D[PERS ? order[it] : it];   // the order is read only by persistent launches
    const int R = d.m + d.k;
    wg_potrf<T, NB, true>(arena + d.front_off, R, R, d.m, R, lds, fail, d.cluster, d.bw);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Banded interior fronts (Eq. 4.2 when M_II has lower bandwidth bw < W and
// the front has at most 64 separator rows, e.g. the finest interiors of a 2D
// grid numbered naturally): one wavefront per front of the list, three parts.
//  1. Band Cholesky of M_II, right-looking one column per step, on a ring of
//     band rows in LDS (a power of two, at least three W-row blocks); band
//     row i is stored by diagonals, ring[i][W-1-r] = A[i][i-r].  Columns of
//     block b+1 are staged before
//     the steps of block b (they hold the rows those steps update), from
//     registers loaded one block ahead.  Each finished column of L_II is
//     written to the front at once (coalesced).
//  2. L_SI = M_SI L_II^{-T}: lane s owns separator row s and keeps its last W
//     values in registers; the coefficients of row j of L_II are LDS
//     broadcasts.
//  3. S = L_SI L_SI^T on the matrix cores, 16 x 16 tiles of the lower
//     triangle accumulated in registers over all blocks; -S is stored once
//     into the front's separator block, which starts at zero (the couplings
//     among separators live in the pair blocks).
// Entries of L_II below the band are neither read nor written.
// ---------------------------------------------------------------------------
constexpr int BE_KMAX = 64;

// Packed factor of a banded front for the apply sweeps, contiguous from
// ElimDesc::pk_off: the band of L_I by diagonals with row stride
// band_pk_ld(m), PB[r][i] = L[i][i-r] and PB[0][i] = 1 / L[i][i] (entries
// with i < r are 0), then, from pk_off + band_pk_lsi(m, bw), L_SI column by
// column, PL[s + j k] = L_SI[s][j].  Both parts start on 64-element bounds.
__host__ __device__ constexpr int band_pk_ld(int m) { return (m + 1) & ~1; }
__host__ __device__ inline int64_t band_pk_lsi(int m, int bw) {
  return (((int64_t)(bw + 1) * band_pk_ld(m)) + 63) & ~(int64_t)63;
}
__host__ __device__ inline int64_t band_pk_elems(int m, int k, int bw) {
  return band_pk_lsi(m, bw) + ((((int64_t)k * m) + 63) & ~(int64_t)63);
}

// Rows of the LDS ring of k_elim_banded<W>: a power of two holding 3W rows,
// so the ring row of band row i is i & (rows - 1).
__host__ __device__ constexpr int be_ring_rows(int w) { return w <= 8 ? 32 : w <= 16 ? 64 : 128; }
__host__ __device__ inline int64_t elim_banded_lds_elems(int w) {
  return (int64_t)be_ring_rows(w) * (w + 1) + (int64_t)BE_KMAX * (w + 1) + WAVE;
}

// Reciprocal and square root of the band pivots: the hardware
// instructions in FP32 (1 ulp, below the rounding of the FP32 factor),
// correctly rounded in FP64.
__device__ __forceinline__ float be_sqrt(float a) { return __builtin_amdgcn_sqrtf(a); }
__device__ __forceinline__ float be_rcp(float a) { return __builtin_amdgcn_rcpf(a); }
__device__ __forceinline__ double be_sqrt(double a) { return sqrt(a); }
__device__ __forceinline__ double be_rcp(double a) { return 1.0 / a; }

template <typename T, int W>
__device__ __forceinline__ void elim_banded_front(const ElimDesc d, T* __restrict__ arena, int* fail,
                                                  T* __restrict__ pk) {
  static_assert(W % 4 == 0 && (W * W) % WAVE == 0, "ring width");
  constexpr int RS = be_ring_rows(W), MASK = RS - 1;
  static_assert(RS >= 3 * W, "ring rows");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* ring = reinterpret_cast<T*>(smem_raw);   // RS rows x W
  T* dinv = ring + RS * W;                    // reciprocal pivots, by ring row (0 beyond m)
  T* tile = dinv + RS;                        // 64 x (W + 1): the block of L_SI, row-major
  T* sink = tile + BE_KMAX * (W + 1);         // one slot per lane for the writes of idle lanes
  typedef typename Mfma<T>::V V;
  const int m = d.m, k = d.k, R = m + k, bw = min(min(d.bw, W - 1), max(m - 1, 0));
  T* C = arena + d.front_off;
  constexpr int E = sizeof(T);
  // every global access of the front and of its packed copy goes through
  // buffer resources (idle lanes pass BUF_OOB; no packed copy: empty range)
  const auto rc = buf_res(C, (int64_t)R * R * E);
  const int lane = threadIdx.x;
  // this lane's pairs (s, t), 1 <= t <= s <= bw, of the trailing update, and
  // the ring columns of A[j+s][j], A[j+t][j] and A[j+s][j+t]; an idle pair
  // (ps = 0) reads a valid entry and writes to the lane's sink slot
  constexpr int NP = (W * (W - 1) / 2 + WAVE - 1) / WAVE;
  int ps[NP], pt[NP], cs[NP], ct[NP], ce[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    int p = lane + q * WAVE, ss = 1;
    while (ss <= bw && p >= ss) p -= ss++;
    ps[q] = ss <= bw ? ss : 0;
    pt[q] = ss <= bw ? p + 1 : 0;
    cs[q] = W - 1 - ps[q];
    ct[q] = W - 1 - pt[q];
    ce[q] = W - 1 - (ps[q] - pt[q]);
  }
  const int sink_off = (int)(sink - ring) + lane;
  // staging: entries A[c + r][c] of the columns c of a block, r = 0..bw
  constexpr int NS = W * W / WAVE;
  auto load_cols = [&](int b, T* v) {
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      const int idx = lane + q * WAVE, c = b * W + idx / W, r = idx % W, i = c + r;
      v[q] = buf_ld(rc, buf_off(r <= bw && c < m && i < m, i + (int64_t)c * R, E), T());
    }
  };
  auto store_cols = [&](int b, const T* v) {
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      const int idx = lane + q * WAVE, c = b * W + idx / W, r = idx % W, i = c + r;
      if (r <= bw && c < m && i < m) ring[(i & MASK) * W + (W - 1 - r)] = v[q];
    }
  };
  // packed copy for the apply (pk_off >= 0): band by diagonals, then L_SI
  const bool packed = d.pk_off >= 0;
  T* PB = pk + (packed ? d.pk_off : 0);
  const auto rp = buf_res(PB, packed ? band_pk_elems(m, k, bw) * E : 0);
  const int64_t lsi0 = band_pk_lsi(m, bw);   // L_SI in the packed copy
  const int pld = band_pk_ld(m);
  // the finished columns of block b (band entries L[c + r][c]) into the front
  // and into the packed band (reciprocal on the diagonal)
  auto store_out = [&](int b) {
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      const int idx = lane + q * WAVE, c = b * W + idx / W, r = idx % W, i = c + r;
      const bool ok = r <= bw && c < m && i < m;
      const T v = ring[(i & MASK) * W + (W - 1 - r)];
      buf_st(rc, buf_off(ok, i + (int64_t)c * R, E), v);
      buf_st(rp, buf_off(ok, (int64_t)r * pld + i, E), r == 0 ? dinv[i & MASK] : v);
    }
    // band entries above the first row of the band (i < r) are zero
    if (b == 0)
      for (int idx = lane; idx < (bw + 1) * bw; idx += WAVE) {
        const int r = 1 + idx / bw, i = idx % bw;
        buf_st(rp, buf_off(i < r && i < m, (int64_t)r * pld + i, E), T(0));
      }
  };
  auto zero_block = [&](int b) {
    for (int idx = lane; idx < W * W; idx += WAVE) ring[((b * W + idx / W) & MASK) * W + idx % W] = T(0);
    if (lane < W) dinv[(b * W + lane) & MASK] = T(0);
  };
  const int nblk = (m + W - 1) / W;
  T pre[NS];
  zero_block(0);
  zero_block(1);
  __builtin_amdgcn_wave_barrier();
  load_cols(0, pre);
  store_cols(0, pre);
  if (nblk > 1) load_cols(1, pre);
  // separator row of this lane: M_SI / L_SI entry (lane, j) at m + lane + j R
  const bool srow = lane < k;
  // mcur: this lane's M_SI row over the current block's columns (loaded
  // for the next block as soon as phase 2 is done with it)
  T x[W], mcur[W];
#pragma unroll
  for (int t = 0; t < W; ++t) {
    x[t] = T(0);
    mcur[t] = buf_ld(rc, buf_off(srow && t < m, m + lane + (int64_t)t * R, E), T());
  }
  constexpr int KT = BE_KMAX / 16, NT = KT * (KT + 1) / 2;
  const int kt = (k + 15) / 16;
  V acc[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[q][v] = T(0);
  T minpiv = T(1);   // smallest pivot seen (a non-positive one is reported once, after the front)
  for (int b = 0; b < nblk; ++b) {
    const int j0 = b * W;
    // stage the columns of block b + 1 (rows of blocks b + 1, b + 2); fetch those of b + 2
    __builtin_amdgcn_wave_barrier();
    if (b + 1 < nblk) {
      zero_block(b + 2);
      __builtin_amdgcn_wave_barrier();
      store_cols(b + 1, pre);
      if (b + 2 < nblk) load_cols(b + 2, pre);
    }
    __builtin_amdgcn_wave_barrier();
    // ---- 1. band Cholesky, columns j0 .. j0 + W - 1 (branch-free: idle lanes
    // read valid entries and write to their sink slot) ----
    const int jend = min(W, m - j0);
    const bool sc0 = lane >= 1 && lane <= bw;   // lane scales A[j + lane][j]
    for (int t = 0; t < jend; ++t) {
      const int j = j0 + t;
      const int dg = (j & MASK) * W + (W - 1);
      T a = ring[dg];
      const int sa = ((j + lane) & MASK) * W + (W - 1 - min(lane, W - 1));
      const T colv = ring[sa];
      T as[NP], at[NP], e[NP];
      int ea[NP];
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        const int rs = ((j + ps[q]) & MASK) * W, rt = ((j + pt[q]) & MASK) * W;
        as[q] = ring[rs + cs[q]];
        at[q] = ring[rt + ct[q]];
        e[q] = ring[rs + ce[q]];
        ea[q] = (ps[q] > 0 && j + ps[q] < m) ? rs + ce[q] : sink_off;
      }
      minpiv = min(minpiv, a);
      a = a > T(0) ? a : T(1);
      const T l = be_sqrt(a), inv = be_rcp(l), inv2 = inv * inv;
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int q = 0; q < NP; ++q) ring[ea[q]] = e[q] - as[q] * at[q] * inv2;
      ring[(sc0 && j + lane < m) ? sa : sink_off] = colv * inv;
      ring[lane == 0 ? dg : sink_off] = l;
      dinv[j & MASK] = inv;
      __builtin_amdgcn_wave_barrier();
    }
    store_out(b);
    // ---- 2. L_SI columns j0 .. j0 + W - 1 (rows beyond m: zero coefficients) ----
#pragma unroll
    for (int t = 0; t < W; ++t) {
      const int j = j0 + t;
      const T* row = ring + (j & MASK) * W;
      T acc2 = mcur[t];
#pragma unroll
      for (int r = W - 1; r >= 1; --r) acc2 -= row[W - 1 - r] * x[(t - r + W) % W];
      x[t] = acc2 * dinv[j & MASK];
      buf_st(rc, buf_off(srow && j < m, m + lane + (int64_t)j * R, E), x[t]);
      buf_st(rp, buf_off(srow && j < m, lsi0 + lane + (int64_t)j * k, E), x[t]);
    }
#pragma unroll
    for (int t = 0; t < W; ++t) {
      const int jn = j0 + W + t;
      mcur[t] = buf_ld(rc, buf_off(srow && jn < m, m + lane + (int64_t)jn * R, E), T());
    }
    // ---- 3. S += L_SI(:, block) L_SI(:, block)^T ----
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int t = 0; t < W; ++t) tile[lane * (W + 1) + t] = x[t];
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int c = 0; c < W / 4; ++c) {
      T op[KT];
#pragma unroll
      for (int X = 0; X < KT; ++X) op[X] = tile[(16 * X + lane % 16) * (W + 1) + 4 * c + lane / 16];
      int q = 0;
#pragma unroll
      for (int I = 0; I < KT; ++I)
#pragma unroll
        for (int J = 0; J <= I; ++J, ++q) acc[q] = Mfma<T>::op(op[I], op[J], acc[q]);
    }
  }
  if (!(minpiv > T(0)) && lane == 0) atomicCAS(fail, -1, d.cluster);
  // the separator block of the front receives -L_SI L_SI^T (lower triangle)
  int q = 0;
#pragma unroll
  for (int I = 0; I < KT; ++I)
#pragma unroll
    for (int J = 0; J <= I; ++J, ++q) {
      if (I >= kt) continue;
      const int col = 16 * J + lane % 16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * I + Mfma<T>::drow(lane, v);
        buf_st(rc, buf_off(row < k && col < k && row >= col, (m + row) + (int64_t)(m + col) * R, E), -acc[q][v]);
      }
    }
}

template <typename T, int W>
__global__ __launch_bounds__(WAVE) void k_elim_banded(const ElimDesc* __restrict__ D, T* __restrict__ arena,
                                                      int* fail, const int32_t* __restrict__ list,
                                                      T* __restrict__ pk) {
  elim_banded_front<T, W>(D[list[blockIdx.x]], arena, fail, pk);
}

// Two ring widths in one launch: the nA fronts of listA (width WA: the few
// wide fronts, e.g. the boundary blocks of a grid) first, so that they are
// dispatched before the many fronts of listB (width WB) take the compute
// units and end about when those do instead of trailing them; registers and
// LDS are those of the wider class.
template <typename T, int WA, int WB>
__global__ __launch_bounds__(WAVE) void k_elim_banded2(const ElimDesc* __restrict__ D, T* __restrict__ arena,
                                                       int* fail, const int32_t* __restrict__ listA, int nA,
                                                       const int32_t* __restrict__ listB, T* __restrict__ pk) {
  if ((int)blockIdx.x < nA) elim_banded_front<T, WA>(D[listA[blockIdx.x]], arena, fail, pk);
  else elim_banded_front<T, WB>(D[listB[blockIdx.x - nA]], arena, fail, pk);
}

// Subtract the interiors' Schur complements from the separator pair blocks,
// contributions summed in ascending interior order.
template <typename T>
__global__ __launch_bounds__(WG) void k_schur(const PairDesc* __restrict__ P, const SchurDesc* __restrict__ S,
                                              const T* __restrict__ fronts, T* __restrict__ blocks) {
  const PairDesc pd = P[blockIdx.x];
  if (pd.c_cnt == 0) return;
  T* blk = blocks + pd.blk_off;
  const int tot = pd.s_a * pd.s_b;
  for (int idx = threadIdx.x; idx < tot; idx += WG) {
    const int i = idx % pd.s_a, j = idx / pd.s_a;
    T acc = blk[idx];
    for (int c = 0; c < pd.c_cnt; ++c) {
      const SchurDesc s = S[pd.c_ptr + c];
      const T* src = fronts + s.src_off;
      if (s.diag) acc += src[max(i, j) + (int64_t)min(i, j) * s.src_ld];
      else acc += src[j + (int64_t)i * s.src_ld];
    }
    blk[idx] = acc;
  }
}

// Compression fronts [M_BB ; M_X1B ; ... ] ((s + K) x s) from the pair blocks.
template <typename T>
__global__ __launch_bounds__(WG) void k_comp_gather(const CompDesc* __restrict__ D, const CompNbr* __restrict__ NB,
                                                    const T* __restrict__ blocks, T* __restrict__ cf) {
  const CompDesc d = D[blockIdx.x];
  const int64_t ld = d.s + d.K;
  T* F = cf + d.cf_off;
  const T* dg = blocks + d.blk_diag;
  for (int idx = threadIdx.x; idx < d.s * d.s; idx += WG) {
    int i = idx % d.s, j = idx / d.s;
    F[i + (int64_t)j * ld] = dg[idx];
  }
  for (int q = 0; q < d.nnb; ++q) {
    const CompNbr x = NB[d.nb_ptr + q];
    const T* b = blocks + x.blk_off;
    for (int idx = threadIdx.x; idx < x.s_x * d.s; idx += WG) {
      int j = idx % x.s_x, i = idx / x.s_x;   // row j of X, column i of B
      T v = x.trans ? b[i + (int64_t)j * d.s] : b[j + (int64_t)i * x.s_x];
      F[(x.row + j) + (int64_t)i * ld] = v;
    }
  }
}

// Householder QR with column pivoting of the s x c matrix N (ld s), stopped
// at the numerical rank (Eq. 3.3; convention shared with the oracle: pivot =
// largest recomputed trailing column norm, near-ties within a relative 1e-10
// to the lowest index; beta = -sign(alpha) ||x||, no reflection for a zero
// tail).  One thread per column for norms and updates, wave 0 forms each
// reflector.  Leaves the reflectors below the diagonal of the first r
// columns, tau[0..r), and returns r.  `nrm` holds c entries of scratch.
// fixed >= 0: exactly min(fixed, s, c) steps instead of the threshold (the
// truncated rank-revealing QR of Eq. 7.5); a step on a zero trailing part
// keeps its column and takes no reflection.
template <typename T>
__device__ int wg_qrcp(T* N, int s, int c, T* nrm, T* tau, double rank_tol, int* sh_int, T* sh_val,
                       int fixed = -1) {
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  for (int j = threadIdx.x; j < c; j += WG) {
    const T* col = N + (int64_t)j * s;
    T acc = 0;
#pragma unroll 8
    for (int i = 0; i < s; ++i) acc += col[i] * col[i];
    nrm[j] = sqrt(acc);
  }
  int r = 0;
  const int kmax = min(s, c);
  for (int k = 0; k < kmax; ++k) {
    __syncthreads();
    if (threadIdx.x == 0) {
      T nmax = 0;
      for (int j = k; j < c; ++j) nmax = nrm[j] > nmax ? nrm[j] : nmax;
      if (k == 0) sh_val[1] = nmax;
      int stop = fixed >= 0 ? (k >= fixed) : ((nmax == T(0)) || (nmax <= (T)rank_tol * sh_val[1]));
      int piv = k;
      if (!stop) {
        const T thr = nmax * (T)(1.0 - TIE_RTOL);
        for (int j = k; j < c; ++j)
          if (nrm[j] >= thr) {
            piv = j;
            break;
          }
        nrm[piv] = nrm[k];
      }
      sh_int[0] = piv;
      sh_int[1] = stop;
    }
    __syncthreads();
    if (sh_int[1]) break;
    const int piv = sh_int[0];
    if (piv != k)
      for (int i = threadIdx.x; i < s; i += WG) {
        const T a = N[i + (int64_t)k * s];
        N[i + (int64_t)k * s] = N[i + (int64_t)piv * s];
        N[i + (int64_t)piv * s] = a;
      }
    __syncthreads();
    if (w == 0) {
      T* x = N + (int64_t)k * s;
      T part = 0;
      for (int i = k + 1 + lane; i < s; i += WAVE) part += x[i] * x[i];
      const T tail = wave_sum(part);
      const T alpha = x[k];
      T beta = alpha, tk = 0, scale = 0;
      if (tail != T(0)) {
        const T nv = sqrt(alpha * alpha + tail);
        beta = alpha >= T(0) ? -nv : nv;
        tk = (beta - alpha) / beta;
        scale = T(1) / (alpha - beta);
      }
      if (tk != T(0))
        for (int i = k + 1 + lane; i < s; i += WAVE) x[i] *= scale;
      if (lane == 0) {
        tau[k] = tk;
        sh_val[0] = beta;
      }
    }
    __syncthreads();
    const T tk = tau[k];
    const T* v = N + (int64_t)k * s;
    for (int j = k + 1 + threadIdx.x; j < c; j += WG) {
      T* y = N + (int64_t)j * s;
      if (tk != T(0)) {
        T acc = y[k];
#pragma unroll 8
        for (int i = k + 1; i < s; ++i) acc += v[i] * y[i];
        acc *= tk;
        y[k] -= acc;
#pragma unroll 8
        for (int i = k + 1; i < s; ++i) y[i] -= acc * v[i];
      }
      T nn = 0;
#pragma unroll 8
      for (int i = k + 1; i < s; ++i) nn += y[i] * y[i];
      nrm[j] = sqrt(nn);
    }
    __syncthreads();
    if (threadIdx.x == 0) N[k + (int64_t)k * s] = sh_val[0];
    ++r;
  }
  __syncthreads();
  return r;
}

// One compression (Eqs. 3.1-3.4): L_B = chol(M_BB), Mhat^T = M_XB L_B^{-T},
// N = [L^T Phi_B | Mhat_X Phi_X ...], pivoted Householder QR of N stopped at
// the numerical rank, and (Q^T L^T Phi_B)[:r] into the Phi scratch.  N is
// kept in LDS when it fits (NLDS), else in its global buffer.
template <typename T, int PNB, bool NLDS, bool PERS>
__global__ __launch_bounds__(WG) void k_compress(const CompDesc* __restrict__ D, const CompNbr* __restrict__ NB,
                                                 T* __restrict__ cf, T* __restrict__ nbuf, T* __restrict__ phi,
                                                 T* __restrict__ ltphi, T* __restrict__ tau_all,
                                                 int* __restrict__ rank, int pi, double rank_tol, int* fail,
                                                 int prefactored, int bf16n, const int32_t* __restrict__ order,
                                                 int n, int* ctr, const int32_t* __restrict__ fixed_rank) {
  // Phi of the neighbours is read here and must not change during the launch.
  // With `prefactored`, L_B and L_B^{-1} M_BX are already in the front.
  // Persistent over the level's separators (costliest first).
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  __shared__ int sh_int[2];
  __shared__ T sh_val[2];
  __shared__ int sh_item;
  for (int round = 0; PERS || round == 0; ++round) {
  const int item = next_item<PERS>(ctr, &sh_item, round, n);
  if (item >= n) break;
  const int ci = PERS ? order[item] : item;
  const CompDesc d = D[ci];
  const int s = d.s, c = d.c;
  const int64_t ld = s + d.K;
  T* F = cf + d.cf_off;
  if (!prefactored) wg_potrf<T, PNB, false>(F, ld, s + d.K, s, s, lds, fail, d.cluster, s);
  __syncthreads();
  T* Ng = nbuf + d.n_off;
  T* nrm = lds;
  T* N = NLDS ? lds + ((c + 3) & ~3) : Ng;
  const T* PhB = phi + d.phi_off;
  T* LtP = ltphi + d.ltphi_off;
  // ---- N (Eq. 4.5): [L^T Phi_B | Mhat_BX Phi_X or Mhat_BX ... | 0] ----------
  for (int idx = threadIdx.x; idx < s * pi; idx += WG) {
    const int i = idx % s, p = idx / s;
    T acc = 0;
#pragma unroll 8
    for (int j = i; j < s; ++j) acc += F[j + (int64_t)i * ld] * PhB[j + (int64_t)p * s];
    if (d.self_cols && !bf16n) N[i + (int64_t)p * s] = acc;
    LtP[i + (int64_t)p * s] = acc;
  }
  // BF16N form: the products of N from bfloat16 operands on the matrix cores
  // (FP32 accumulation), 16-row tiles of every block dealt to the wavefronts
  if (bf16n && pi <= 16) {
    const int wv = threadIdx.x / WAVE, nt = (s + 15) / 16;
    int task = 0;
    if (d.self_cols)
      for (int t = 0; t < nt; ++t, ++task)
        if (task % (WG / WAVE) == wv)
          wave_bf16_tile<T>(16 * t, s, pi, s, [&](int i, int j) { return j >= i ? F[j + (int64_t)i * ld] : T(0); },
                            [&](int j, int p) { return PhB[j + (int64_t)p * s]; }, N, s);
    for (int q = 0; q < d.nnb; ++q) {
      const CompNbr x = NB[d.nb_ptr + q];
      if (x.full) continue;
      const T* PhX = phi + x.phi_off;
      for (int t = 0; t < nt; ++t, ++task)
        if (task % (WG / WAVE) == wv)
          wave_bf16_tile<T>(16 * t, s, pi, x.s_x, [&](int i, int j) { return F[(x.row + j) + (int64_t)i * ld]; },
                            [&](int j, int p) { return PhX[j + (int64_t)p * x.s_x]; }, N + (int64_t)x.col * s, s);
    }
  } else if (bf16n && d.self_cols) {
    for (int idx = threadIdx.x; idx < s * pi; idx += WG) {
      const int i = idx % s, p = idx / s;
      T acc16 = 0;
      for (int j = i; j < s; ++j) acc16 += bf16_round(F[j + (int64_t)i * ld]) * bf16_round(PhB[j + (int64_t)p * s]);
      N[i + (int64_t)p * s] = acc16;
    }
  }
  int cend = d.self_cols;
  for (int q = 0; q < d.nnb; ++q) {
    const CompNbr x = NB[d.nb_ptr + q];
    if (x.full) {
      for (int idx = threadIdx.x; idx < s * x.s_x; idx += WG) {
        const int i = idx % s, j = idx / s;
        const T v = F[(x.row + j) + (int64_t)i * ld];
        N[i + (int64_t)(x.col + j) * s] = bf16n ? bf16_round(v) : v;
      }
      cend = x.col + x.s_x;
      continue;
    }
    const T* PhX = phi + x.phi_off;
    if (!(bf16n && pi <= 16))
      for (int idx = threadIdx.x; idx < s * pi; idx += WG) {
        const int i = idx % s, p = idx / s;
        T acc = 0;
        if (bf16n)
          for (int j = 0; j < x.s_x; ++j)
            acc += bf16_round(F[(x.row + j) + (int64_t)i * ld]) * bf16_round(PhX[j + (int64_t)p * x.s_x]);
        else
#pragma unroll 8
          for (int j = 0; j < x.s_x; ++j) acc += F[(x.row + j) + (int64_t)i * ld] * PhX[j + (int64_t)p * x.s_x];
        N[i + (int64_t)(x.col + p) * s] = acc;
      }
    cend = x.col + pi;
  }
  for (int idx = threadIdx.x; idx < s * (c - cend); idx += WG) N[(int64_t)cend * s + idx] = T(0);
  __syncthreads();
  // ---- pivoted Householder QR of N (Eq. 3.3) ---------------------------------
  T* tau = tau_all + d.tau_off;
  const int r = wg_qrcp(N, s, c, nrm, tau, rank_tol, sh_int, sh_val, fixed_rank ? fixed_rank[ci] : -1);
  if (NLDS)
    for (int idx = threadIdx.x; idx < s * r; idx += WG) Ng[idx] = N[idx];
  // ---- (Q^T L^T Phi_B)[:r] (Eq. 3.4) into the scratch; neighbours may still be
  // reading Phi_B, so k_phi_commit installs it after every compression ended.
  if (r < s) wg_apply_qt(N, s, tau, s, r, LtP, s, pi);
  if (threadIdx.x == 0) rank[ci] = r;
  __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Compression of a small separator (s <= 64 rows, c <= 128 columns of N) by
// one wavefront, the same steps and conventions as k_compress (Eqs. 3.1-3.4,
// 4.5; pivot = largest recomputed column norm, near-ties to the lowest index,
// stop at rank_tol relative to the first pivot norm): the front, the Phi
// blocks and N are staged in LDS once, so the sequential parts wait on LDS
// instead of device memory and need no workgroup barriers.  Lane i owns row
// i of M_BB in registers for its Cholesky and row i of the neighbour part for
// L_B^{-1}; in the pivoted QR lane j owns columns j and j + 64 (their norms),
// the pivot is found with a wave maximum and a ballot.
// ---------------------------------------------------------------------------
constexpr int CS_SMAX = 64, CS_CMAX = 128;

__host__ __device__ inline int64_t comp_small_lds_elems(int s, int K, int c, int pi) {
  const int R = s + K;
  return (int64_t)(R | 1) * s + (int64_t)(s | 1) * c + (int64_t)R * pi + (int64_t)s * pi + s + c +
         (int64_t)(s | 1) * s;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    const T u = __shfl_xor(v, o, WAVE);
    v = u > v ? u : v;
  }
  return v;
}

// Copy of n contiguous device elements into LDS by the first NT threads (one
// wavefront by default) with U loads in flight per thread (buffer loads over
// exactly the n elements, so the threads past the end load nothing): element
// e goes to dst[dl(e)].
template <typename T, int U = 8, int NT = WAVE, typename DL>
__device__ __forceinline__ void wave_stage(T* dst, const T* src, int n, DL dl) {
  const __amdgpu_buffer_rsrc_t r = buf_res(src, (int64_t)n * (int64_t)sizeof(T));
  const int t = threadIdx.x % NT;
  for (int b = 0; b < n; b += U * NT) {
    T v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = b + u * NT + t;
      v[u] = buf_ld(r, buf_off(e < n, e, (int)sizeof(T)), T());
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = b + u * NT + t;
      if (e < n) dst[dl(e)] = v[u];
    }
  }
}

template <typename T, int NB, int NW>
__global__ __launch_bounds__(NW * WAVE) void k_compress_small(const CompDesc* __restrict__ D,
                                                         const CompNbr* __restrict__ NBR, T* __restrict__ cf,
                                                         T* __restrict__ nbuf, const T* __restrict__ phi,
                                                         T* __restrict__ ltphi, T* __restrict__ tau_all,
                                                         int* __restrict__ rank, int pi, double rank_tol, int* fail,
                                                         int prefactored, int bf16n, T* __restrict__ tb,
                                                         const T* __restrict__ blocks,
                                                         const int32_t* __restrict__ fixed_rank) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int ci = blockIdx.x;
  const CompDesc d = D[ci];
  const int s = d.s, K = d.K, c = d.c, R = s + K;
  const int ldf = R | 1, ldn = s | 1;
  T* Fl = reinterpret_cast<T*>(smem_raw);   // R x s, ld ldf
  T* Nl = Fl + (int64_t)ldf * s;            // s x c, ld ldn
  T* Ph = Nl + (int64_t)ldn * c;            // R x pi, ld R: Phi_B in rows [0, s), Phi_X at the neighbour's front rows
  T* Lt = Ph + (int64_t)R * pi;             // s x pi, ld s
  T* invd = Lt + (int64_t)s * pi;           // s reciprocal pivots
  T* taul = invd + s;                       // c reflector coefficients
  T* Xl = taul + c;                         // s x s, ld s | 1: T_B = Q^T L_B^{-1}
  // NW wavefronts: all of them in the parallel phases (staging, neighbour
  // rows, write-back, N, the reflector pass), wavefront 0 alone in the
  // sequential ones (Cholesky, QRCP); each element is computed by the same
  // code whatever NW is, so the values do not depend on it
  constexpr int NT = NW * WAVE;
  const int tid = threadIdx.x, lane = tid % WAVE, w = tid / WAVE;
  __shared__ int sh_r;
  auto sync = [] {
    if constexpr (NW > 1) __syncthreads();
    else __builtin_amdgcn_wave_barrier();
  };
  T* F = cf + d.cf_off;
  // ---- stage the front and the Phi blocks ----
  // (every block is read in its own storage order, batches of loads in flight)
  if (blocks) {
    // the front straight from the pair blocks (what k_comp_gather puts in cf):
    // M_BB, then M_XB of every neighbour X (stored as M_BX when trans)
    wave_stage<T, 8, NT>(Fl, blocks + d.blk_diag, s * s, [&](int e) { return e % s + (e / s) * ldf; });
    for (int q = 0; q < d.nnb; ++q) {
      const CompNbr x = NBR[d.nb_ptr + q];
      const int sx = x.s_x, xr = x.row;
      if (x.trans)   // M_BX: element e is row e % s of B, column e / s of X
        wave_stage<T, 8, NT>(Fl, blocks + x.blk_off, sx * s, [&](int e) { return xr + e / s + (e % s) * ldf; });
      else           // M_XB: element e is row e % s_X of X, column e / s_X of B
        wave_stage<T, 8, NT>(Fl, blocks + x.blk_off, sx * s, [&](int e) { return xr + e % sx + (e / sx) * ldf; });
    }
  } else {
    wave_stage<T, 8, NT>(Fl, F, R * s, [&](int e) { return e % R + (e / R) * ldf; });
  }
  wave_stage<T, 8, NT>(Ph, phi + d.phi_off, s * pi, [&](int e) { return e % s + (e / s) * R; });
  for (int q = 0; q < d.nnb; ++q) {
    const CompNbr x = NBR[d.nb_ptr + q];
    if (x.full) continue;
    const int sx = x.s_x, xr = x.row;
    wave_stage<T, 8, NT>(Ph, phi + x.phi_off, sx * pi, [&](int e) { return xr + e % sx + (e / sx) * R; });
  }
  sync();
  if (!prefactored) {
    // ---- L_B = chol(M_BB): lane i keeps row i in registers ----
    if (w == 0) {
    T a[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) a[k] = (lane < s && k < s && k <= lane) ? Fl[lane + k * ldf] : T(0);
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      if (j < s) {
        T dd = lane_bcast(a[j], j);
        if (!(dd > T(0))) {
          if (lane == 0) atomicCAS(fail, -1, d.cluster);
          dd = T(1);
        }
        const T sd = sqrt(dd), inv = T(1) / sd;
        const T l = (lane == j) ? sd : a[j] * inv;
        if (lane >= j) a[j] = l;
        if (lane == j) invd[j] = inv;
#pragma unroll
        for (int k = j + 1; k < NB; ++k) {
          const T lk = lane_bcast(l, k);
          if (lane >= k) a[k] -= l * lk;
        }
      }
    }
    if (lane < s)
#pragma unroll
      for (int k = 0; k < NB; ++k)
        if (k < s && k <= lane) Fl[lane + k * ldf] = a[k];
    }
    sync();
    // ---- neighbour rows: row <- row L_B^{-T}, one row per lane, the row's
    // solved entries in registers (the coefficients of L_B are LDS
    // broadcasts) ----
    for (int i = s + tid; i < R; i += NT) {
      T x[NB];
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        if (j < s) {
          T acc = Fl[i + j * ldf];
#pragma unroll
          for (int p = 0; p < j; ++p) acc -= x[p] * Fl[j + p * ldf];
          x[j] = acc * invd[j];
        }
      }
#pragma unroll
      for (int j = 0; j < NB; ++j)
        if (j < s) Fl[i + j * ldf] = x[j];
    }
    sync();
    // the factored front to cf (all of it when the staging skipped cf, so
    // that cf holds what the gather and this write-back would have left)
    for (int idx = tid; idx < R * s; idx += NT) {
      const int i = idx % R, j = idx / R;
      if (i >= j || blocks) F[idx] = Fl[i + j * ldf];
    }
  }
  // ---- N (Eq. 4.5) and L^T Phi_B ----
  for (int idx = tid; idx < s * pi; idx += NT) {
    const int i = idx % s, p = idx / s;
    T acc = 0;
#pragma unroll 8
    for (int j = i; j < s; ++j) acc += Fl[j + i * ldf] * Ph[j + p * R];
    if (d.self_cols && !bf16n) Nl[i + p * ldn] = acc;
    Lt[i + p * s] = acc;
  }
  // BF16N form: the products of N from bfloat16 operands on the matrix cores
  // (FP32 accumulation); pi <= 16 columns per block
  const bool mma = bf16n && pi <= 16;
  if (bf16n && d.self_cols) {
    if (mma) {
      if (w == 0)
        wave_bf16_gemm<T>(s, pi, s, [&](int i, int j) { return j >= i ? Fl[j + i * ldf] : T(0); },
                          [&](int j, int p) { return Ph[j + p * R]; }, Nl, ldn);
    } else {
      for (int idx = tid; idx < s * pi; idx += NT) {
        const int i = idx % s, p = idx / s;
        T acc16 = 0;
        for (int j = i; j < s; ++j) acc16 += bf16_round(Fl[j + i * ldf]) * bf16_round(Ph[j + p * R]);
        Nl[i + p * ldn] = acc16;
      }
    }
  }
  int cend = d.self_cols;
  for (int q = 0; q < d.nnb; ++q) {
    const CompNbr x = NBR[d.nb_ptr + q];
    if (x.full) {
      for (int idx = tid; idx < s * x.s_x; idx += NT) {
        const int i = idx % s, j = idx / s;
        const T v = Fl[(x.row + j) + i * ldf];
        Nl[i + (x.col + j) * ldn] = bf16n ? bf16_round(v) : v;
      }
      cend = x.col + x.s_x;
      continue;
    }
    if (mma) {
      const int xr = x.row;
      if (w == 0)
        wave_bf16_gemm<T>(s, pi, x.s_x, [&](int i, int j) { return Fl[(xr + j) + i * ldf]; },
                          [&](int j, int p) { return Ph[(xr + j) + p * R]; }, Nl + x.col * ldn, ldn);
    } else {
      for (int idx = tid; idx < s * pi; idx += NT) {
        const int i = idx % s, p = idx / s;
        T acc = 0;
        if (bf16n)
          for (int j = 0; j < x.s_x; ++j)
            acc += bf16_round(Fl[(x.row + j) + i * ldf]) * bf16_round(Ph[(x.row + j) + p * R]);
        else
#pragma unroll 8
          for (int j = 0; j < x.s_x; ++j) acc += Fl[(x.row + j) + i * ldf] * Ph[(x.row + j) + p * R];
        Nl[i + (x.col + p) * ldn] = acc;
      }
    }
    cend = x.col + pi;
  }
  for (int idx = tid; idx < s * (c - cend); idx += NT) Nl[idx % s + (cend + idx / s) * ldn] = T(0);
  sync();
  // ---- pivoted Householder QR of N (Eq. 3.3), wavefront 0 ----
  int r = 0;
  if (w == 0) {
  T nr[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int j = lane + h * WAVE;
    T acc = 0;
    if (j < c)
#pragma unroll 8
      for (int i = 0; i < s; ++i) acc += Nl[i + j * ldn] * Nl[i + j * ldn];
    nr[h] = sqrt(acc);
  }
  T ref = 0;
  const int kmax = min(s, c);
  const int fixed = fixed_rank ? fixed_rank[ci] : -1;
  for (int k = 0; k < kmax; ++k) {
    const T m0 = (lane >= k && lane < c) ? nr[0] : T(0);
    const T m1 = (lane + WAVE >= k && lane + WAVE < c) ? nr[1] : T(0);
    const T nmax = wave_max(m0 > m1 ? m0 : m1);
    if (k == 0) ref = nmax;
    if (fixed >= 0 ? k >= fixed : (nmax == T(0) || nmax <= (T)rank_tol * ref)) break;
    const T thr = nmax * (T)(1.0 - TIE_RTOL);
    const unsigned long long b0 = __ballot(lane >= k && lane < c && nr[0] >= thr);
    const unsigned long long b1 = __ballot(lane + WAVE >= k && lane + WAVE < c && nr[1] >= thr);
    const int piv = b0 ? __ffsll((long long)b0) - 1 : WAVE + __ffsll((long long)b1) - 1;
    const T nk = k < WAVE ? lane_bcast(nr[0], k) : lane_bcast(nr[1], k - WAVE);
    if (piv < WAVE) {
      if (lane == piv) nr[0] = nk;
    } else if (lane == piv - WAVE) {
      nr[1] = nk;
    }
    if (piv != k)
      for (int i = lane; i < s; i += WAVE) {
        const T t0 = Nl[i + k * ldn];
        Nl[i + k * ldn] = Nl[i + piv * ldn];
        Nl[i + piv * ldn] = t0;
      }
    __builtin_amdgcn_wave_barrier();
    const T xi = lane < s ? Nl[lane + k * ldn] : T(0);
    const T tail = wave_sum((lane > k && lane < s) ? xi * xi : T(0));
    const T alpha = lane_bcast(xi, k);
    T beta = alpha, tk = 0, scale = 0;
    if (tail != T(0)) {
      const T nv = sqrt(alpha * alpha + tail);
      beta = alpha >= T(0) ? -nv : nv;
      tk = (beta - alpha) / beta;
      scale = T(1) / (alpha - beta);
    }
    if (tk != T(0) && lane > k && lane < s) Nl[lane + k * ldn] = xi * scale;
    if (lane == 0) taul[k] = tk;
    __builtin_amdgcn_wave_barrier();
    const T* v = Nl + k * ldn;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int j = lane + h * WAVE;
      if (j > k && j < c) {
        T* y = Nl + j * ldn;
        // the updated column's trailing norm is summed in the update pass
        // (the same values in the same order as a pass of its own)
        T nn = 0;
        if (tk != T(0)) {
          T acc = y[k];
#pragma unroll 8
          for (int i = k + 1; i < s; ++i) acc += v[i] * y[i];
          acc *= tk;
          y[k] -= acc;
#pragma unroll 8
          for (int i = k + 1; i < s; ++i) {
            const T yi = y[i] - acc * v[i];
            y[i] = yi;
            nn += yi * yi;
          }
        } else {
#pragma unroll 8
          for (int i = k + 1; i < s; ++i) nn += y[i] * y[i];
        }
        nr[h] = sqrt(nn);
      }
    }
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) Nl[k + k * ldn] = beta;
    ++r;
  }
  __builtin_amdgcn_wave_barrier();
  if (lane == 0) sh_r = r;
  }
  sync();
  if constexpr (NW > 1) r = sh_r;
  // ---- reflectors, tau and the rank out; then Q^T acts, one column per
  // lane, on the columns of L_B^{-1} (T_B = Q^T L_B^{-1}, for the apply and
  // the coarse couplings) and on those of L^T Phi_B ((Q^T L^T Phi_B)[:r],
  // Eq. 3.4); the column in registers, the coefficients of L_B and of the
  // reflectors LDS broadcasts ----
  T* Ng = nbuf + d.n_off;
  for (int idx = tid; idx < s * r; idx += NT) Ng[idx] = Nl[idx % s + (idx / s) * ldn];
  T* tau = tau_all + d.tau_off;
  for (int k = tid; k < r; k += NT) tau[k] = taul[k];
  if (r < s) {
    const int ldx = s | 1;
    for (int j = tid; j < s + pi; j += NT) {
      T x[NB];
      if (j < s) {
        // column j of L_B^{-1}: rows above j are zero, and the products with
        // them that the unrolled solve adds are zeros
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          if (i < s) {
            T acc = i == j ? T(1) : T(0);
#pragma unroll
            for (int p = 0; p < i; ++p) acc -= Fl[i + p * ldf] * x[p];
            x[i] = i < j ? T(0) : acc / Fl[i + i * ldf];
          }
        }
      } else {
        const T* lc = Lt + (j - s) * s;
#pragma unroll
        for (int i = 0; i < NB; ++i)
          if (i < s) x[i] = lc[i];
      }
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        if (k < r) {
          const T tk = taul[k];
          if (tk != T(0)) {
            T acc = x[k];
#pragma unroll
            for (int i = k + 1; i < NB; ++i)
              if (i < s) acc += Nl[i + k * ldn] * x[i];
            acc *= tk;
            x[k] -= acc;
#pragma unroll
            for (int i = k + 1; i < NB; ++i)
              if (i < s) x[i] -= acc * Nl[i + k * ldn];
          }
        }
      }
      T* xc = j < s ? Xl + j * ldx : Lt + (j - s) * s;
#pragma unroll
      for (int i = 0; i < NB; ++i)
        if (i < s) xc[i] = x[i];
    }
    sync();
    T* X = tb + d.tb_off;
    for (int idx = tid; idx < s * s; idx += NT) X[idx] = Xl[idx % s + (idx / s) * ldx];
  }
  T* LtP = ltphi + d.ltphi_off;
  for (int idx = tid; idx < s * pi; idx += NT) LtP[idx] = Lt[idx];
  if (tid == 0) rank[ci] = r;
}

// Phi_B <- (Q^T L^T Phi_B)[:r] for the separators that were compressed.
template <typename T>
__global__ __launch_bounds__(WG) void k_phi_commit(const CompDesc* __restrict__ D, const int* __restrict__ rank,
                                                   const T* __restrict__ ltphi, T* __restrict__ phi, int pi) {
  const CompDesc d = D[blockIdx.x];
  const int r = rank[blockIdx.x];
  if (r >= d.s) return;
  for (int idx = threadIdx.x; idx < r * pi; idx += WG) {
    int i = idx % r, p = idx / r;
    phi[d.phi_off + i + (int64_t)p * d.s] = ltphi[d.ltphi_off + i + (int64_t)p * d.s];
  }
}

// k_pair with one wavefront per pair, PPB pairs per workgroup and the
// intermediate T_a M_ab in LDS (gmax elements per wavefront): the same
// products in the same order, for levels of many small pairs.
constexpr int PPB = 4;
template <typename T>
__global__ __launch_bounds__(PPB * WAVE) void k_pair_w(const PairDesc* __restrict__ P,
                                                       const int32_t* __restrict__ active, int nact,
                                                       const int* __restrict__ rank,
                                                       const int64_t* __restrict__ t_of_comp,
                                                       const T* __restrict__ tb, T* __restrict__ blocks, int gmax) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int q = blockIdx.x * PPB + w;
  if (q >= nact) return;
  const PairDesc pd = P[active[q]];
  const int sa = pd.s_a, sb = pd.s_b;
  const int ra = (pd.ca >= 0 && rank[pd.ca] < sa) ? rank[pd.ca] : sa;
  const int rb = (pd.cb >= 0 && rank[pd.cb] < sb) ? rank[pd.cb] : sb;
  const bool ca = ra < sa, cb = rb < sb;
  T* blk = blocks + pd.blk_off;
  if (pd.a == pd.b) {
    if (ca)
      for (int idx = lane; idx < ra * ra; idx += WAVE) {
        const int i = idx % ra, j = idx / ra;
        blk[i + (int64_t)j * sa] = (i == j) ? T(1) : T(0);
      }
    return;
  }
  T* G = reinterpret_cast<T*>(smem_raw) + (int64_t)w * gmax;   // ra x sb, ld ra
  if (ca) {
    const T* Ta = tb + t_of_comp[pd.ca];
    for (int idx = lane; idx < ra * sb; idx += WAVE) {
      const int i = idx % ra, j = idx / ra;
      T acc = 0;
#pragma unroll 8
      for (int p = 0; p < sa; ++p) acc += Ta[i + (int64_t)p * sa] * blk[p + (int64_t)j * sa];
      G[idx] = acc;
    }
  } else {
    for (int idx = lane; idx < ra * sb; idx += WAVE) G[idx] = blk[(idx % ra) + (int64_t)(idx / ra) * sa];
  }
  // G is written and read by this wavefront only: its LDS accesses are
  // performed in order, the barrier keeps the compiler from moving them
  __builtin_amdgcn_wave_barrier();
  if (cb) {
    const T* Tb = tb + t_of_comp[pd.cb];
    for (int idx = lane; idx < ra * rb; idx += WAVE) {
      const int i = idx % ra, j = idx / ra;
      T acc = 0;
#pragma unroll 8
      for (int r = 0; r < sb; ++r) acc += G[i + (int64_t)r * ra] * Tb[j + (int64_t)r * sb];
      blk[i + (int64_t)j * sa] = acc;
    }
  } else {
    for (int idx = lane; idx < ra * sb; idx += WAVE) blk[(idx % ra) + (int64_t)(idx / ra) * sa] = G[idx];
  }
}

// Coarse couplings C_ab = T_a M_ab T_b^T (the first r rows of T = Q^T L^{-1}
// for a compressed separator, T = I otherwise); the diagonal block of a
// compressed separator becomes I_r (Sec. 3.2: scaled and rotated, fine rows
// dropped).  Two small products through the pair's scratch; launched only
// for pairs that touch a compressed separator.
template <typename T>
__global__ __launch_bounds__(WG) void k_pair(const PairDesc* __restrict__ P, const int32_t* __restrict__ active,
                                             const int* __restrict__ rank, const int64_t* __restrict__ t_of_comp,
                                             const T* __restrict__ tb, T* __restrict__ blocks,
                                             T* __restrict__ scratch) {
  const PairDesc pd = P[active[blockIdx.x]];
  const int sa = pd.s_a, sb = pd.s_b;
  const int ra = (pd.ca >= 0 && rank[pd.ca] < sa) ? rank[pd.ca] : sa;
  const int rb = (pd.cb >= 0 && rank[pd.cb] < sb) ? rank[pd.cb] : sb;
  const bool ca = ra < sa, cb = rb < sb;
  T* blk = blocks + pd.blk_off;
  if (pd.a == pd.b) {
    if (ca)
      for (int idx = threadIdx.x; idx < ra * ra; idx += WG) {
        const int i = idx % ra, j = idx / ra;
        blk[i + (int64_t)j * sa] = (i == j) ? T(1) : T(0);
      }
    return;
  }
  T* G = scratch + pd.scratch_off;   // ra x sb, ld ra
  if (ca) {
    const T* Ta = tb + t_of_comp[pd.ca];
    for (int idx = threadIdx.x; idx < ra * sb; idx += WG) {
      const int i = idx % ra, j = idx / ra;
      T acc = 0;
#pragma unroll 8
      for (int p = 0; p < sa; ++p) acc += Ta[i + (int64_t)p * sa] * blk[p + (int64_t)j * sa];
      G[idx] = acc;
    }
  } else {
    for (int idx = threadIdx.x; idx < ra * sb; idx += WG) G[idx] = blk[(idx % ra) + (int64_t)(idx / ra) * sa];
  }
  __syncthreads();
  if (cb) {
    const T* Tb = tb + t_of_comp[pd.cb];
    for (int idx = threadIdx.x; idx < ra * rb; idx += WG) {
      const int i = idx % ra, j = idx / ra;
      T acc = 0;
#pragma unroll 8
      for (int q = 0; q < sb; ++q) acc += G[i + (int64_t)q * ra] * Tb[j + (int64_t)q * sb];
      blk[i + (int64_t)j * sa] = acc;
    }
  } else {
    for (int idx = threadIdx.x; idx < ra * sb; idx += WG) blk[(idx % ra) + (int64_t)(idx / ra) * sa] = G[idx];
  }
}

// ---------------------------------------------------------------------------
// Apply kernels (Sec. 4.7) and the product form (Sec. 2.1)
// ---------------------------------------------------------------------------

// y (m) <- L^{-1} y in LDS, L lower with ld, blocks of 64 solved by wave 0.
template <typename T>
__device__ void wg_trsv_lower(const T* __restrict__ L, int64_t ld, int m, T* ys) {
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  for (int jb = 0; jb < m; jb += WAVE) {
    const int nb = min(WAVE, m - jb);
    if (w == 0) {
      T v = lane < nb ? ys[jb + lane] : T(0);
      for (int j = 0; j < nb; ++j) {
        T xj = __shfl(v, j, WAVE) / L[(jb + j) + (int64_t)(jb + j) * ld];
        if (lane == j) v = xj;
        if (lane > j && lane < nb) v -= L[(jb + lane) + (int64_t)(jb + j) * ld] * xj;
      }
      if (lane < nb) ys[jb + lane] = v;
    }
    __syncthreads();
    for (int i = jb + nb + threadIdx.x; i < m; i += WG) {
      T acc = 0;
#pragma unroll 8
      for (int j = 0; j < nb; ++j) acc += L[i + (int64_t)(jb + j) * ld] * ys[jb + j];
      ys[i] -= acc;
    }
    __syncthreads();
  }
}

// y (m) <- L^{-T} y in LDS.
template <typename T>
__device__ void wg_trsv_lower_t(const T* __restrict__ L, int64_t ld, int m, T* ys) {
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int nblk = (m + WAVE - 1) / WAVE;
  for (int bj = nblk - 1; bj >= 0; --bj) {
    const int jb = bj * WAVE, nb = min(WAVE, m - jb), below = jb + nb;
    // y_J -= L[below:, J]^T y[below:]
    for (int j = jb + w; j < below; j += WG / WAVE) {
      T acc = 0;
      for (int i = below + lane; i < m; i += WAVE) acc += L[i + (int64_t)j * ld] * ys[i];
      acc = wave_sum(acc);
      if (lane == 0) ys[j] -= acc;
    }
    __syncthreads();
    if (w == 0) {
      T v = lane < nb ? ys[jb + lane] : T(0);
      for (int j = nb - 1; j >= 0; --j) {
        T xj = __shfl(v, j, WAVE) / L[(jb + j) + (int64_t)(jb + j) * ld];
        if (lane == j) v = xj;
        if (lane < j) v -= L[(jb + j) + (int64_t)(jb + lane) * ld] * xj;
      }
      if (lane < nb) ys[jb + lane] = v;
    }
    __syncthreads();
  }
}

// Forward step of one interior: y_I <- L^{-1} y_I, t <- W^T y_I (to scratch).
// mode 1 (product form): y_I <- L y_I, t <- W^T y_I (before the multiply).
template <typename T>
__global__ __launch_bounds__(WG) void k_elim_fwd(const ElimDesc* __restrict__ D, const T* __restrict__ arena,
                                                 const int32_t* __restrict__ slots, T* __restrict__ y, int64_t ldy,
                                                 T* __restrict__ tscr, int64_t ldt, int mode) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* ys = reinterpret_cast<T*>(smem_raw);
  const ElimDesc d = D[blockIdx.x];
  const int m = d.m, k = d.k;
  const int64_t R = (int64_t)m + k;
  const T* C = arena + d.front_off;
  T* yv = y + blockIdx.y * ldy;
  const int32_t* sl = slots + d.slot_off;
  for (int i = threadIdx.x; i < m; i += WG) ys[i] = yv[sl[i]];
  __syncthreads();
  if (mode == 0) wg_trsv_lower(C, R, m, ys);
  T* tv = tscr + blockIdx.y * ldt + d.t_off;
  for (int a = threadIdx.x; a < k; a += WG) {
    T acc = 0;
    for (int j = 0; j < m; ++j) acc += C[(m + a) + (int64_t)j * R] * ys[j];
    tv[a] = acc;
  }
  if (mode == 1) {
    __syncthreads();
    for (int i = threadIdx.x; i < m; i += WG) {
      T acc = 0;
      for (int j = 0; j <= i; ++j) acc += C[i + (int64_t)j * R] * ys[j];
      yv[sl[i]] = acc;
    }
  } else {
    for (int i = threadIdx.x; i < m; i += WG) yv[sl[i]] = ys[i];
  }
}

// y_S <- y_S + sign * sum_I t_I[S part], interiors in ascending order.
template <typename T>
__global__ __launch_bounds__(WG) void k_sepacc(const SepAcc* __restrict__ A, const int64_t* __restrict__ src,
                                               const int32_t* __restrict__ slots, const T* __restrict__ tscr,
                                               int64_t ldt, T* __restrict__ y, int64_t ldy, T sign) {
  const SepAcc a = A[blockIdx.x];
  T* yv = y + blockIdx.y * ldy;
  const T* tv = tscr + blockIdx.y * ldt;
  for (int i = threadIdx.x; i < a.s; i += WG) {
    int32_t sl = slots[a.slot_off + i];
    T acc = 0;
    for (int c = 0; c < a.c_cnt; ++c) acc += tv[src[a.c_ptr + c] + i];
    yv[sl] += sign * acc;
  }
}

// k_sepacc_comp for a separator of at most SB <= 64 rows: wavefront 0 loads
// row i of T_S (registers, zero past s, so its products past s add zeros),
// the contributions and y before its first wait; the arithmetic is that of
// the general path (dynamic LDS: at least 64 entries of ys).
template <typename T, int SB>
__device__ __forceinline__ void sepacc_comp_small(const SepAcc& a, int ci, const int64_t* __restrict__ src,
                                                  const int32_t* __restrict__ sl, const T* __restrict__ tscr,
                                                  T* __restrict__ y, const CompApply* __restrict__ CA,
                                                  const T* __restrict__ tb, T* ys) {
  constexpr int E = sizeof(T);
  const int s = a.s, i = threadIdx.x, ic = min(i, s - 1);
  const bool on = i < s, w0 = threadIdx.x < WAVE;
  int32_t si = 0;
  T xr[SB], v = T(0);
  if (w0) {
    si = sl[ic];
    if (ci >= 0) {
      const auto rx = buf_res(tb + CA[ci].t_off, (int64_t)s * s * E);
#pragma unroll
      for (int j = 0; j < SB; ++j) xr[j] = buf_ld(rx, buf_off(on && j < s, i + (int64_t)j * s, E), T());
    }
    T acc = 0;
    for (int c = 0; c < a.c_cnt; ++c) acc += tscr[src[a.c_ptr + c] + ic];
    v = y[si] + T(-1) * acc;
  }
  if (ci < 0) {   // the same for the whole workgroup
    if (w0 && on) y[si] = v;
    return;
  }
  if (w0) ys[i] = on ? v : T(0);
  __syncthreads();
  if (w0 && on) {
    T o = 0;
#pragma unroll
    for (int j = 0; j < SB; ++j) o += xr[j] * ys[j];
    y[si] = o;
  }
}

// The forward separator step of one level with one right-hand side, one
// workgroup per accumulated separator: y_S <- y_S - sum_I t_I[S part] (as
// k_sepacc with sign -1), then, when S was compressed (cap[b] >= 0),
// y_S <- T_S y_S (as k_comp_apply_t, mode 0) on the values just formed.
// Same arithmetic as the two launches it replaces.  Dynamic LDS: 2 s_max
// (at least 2 x 64 with SB > 0).
template <typename T, int SB>
__global__ __launch_bounds__(WG) void k_sepacc_comp(const SepAcc* __restrict__ A, const int64_t* __restrict__ src,
                                                    const int32_t* __restrict__ slots, const T* __restrict__ tscr,
                                                    T* __restrict__ y, const int32_t* __restrict__ cap,
                                                    const CompApply* __restrict__ CA, const T* __restrict__ tb) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const SepAcc a = A[blockIdx.x];
  const int ci = cap[blockIdx.x];
  T* ys = reinterpret_cast<T*>(smem_raw);
  T* out = ys + a.s;
  const int32_t* sl = slots + a.slot_off;
  // SB > 0: the level's separators have at most SB rows (one register row
  // per thread); 0: the general path only
  if (SB > 0 && a.s <= SB) {
    sepacc_comp_small<T, (SB > 0 ? SB : 16)>(a, ci, src, sl, tscr, y, CA, tb, ys);
    return;
  }
  for (int i = threadIdx.x; i < a.s; i += WG) {
    T acc = 0;
    for (int c = 0; c < a.c_cnt; ++c) acc += tscr[src[a.c_ptr + c] + i];
    T& yi = y[sl[i]];
    const T v = yi + T(-1) * acc;
    if (ci < 0) yi = v;
    else ys[i] = v;
  }
  if (ci < 0) return;
  __syncthreads();
  const int s = a.s;
  const T* X = tb + CA[ci].t_off;
  for (int i = threadIdx.x; i < s; i += WG) {
    T acc = 0;
#pragma unroll 8
    for (int j = 0; j < s; ++j) acc += X[i + (int64_t)j * s] * ys[j];
    out[i] = acc;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < s; i += WG) y[sl[i]] = out[i];
}

// Backward step of one interior: y_I <- L^{-T} (y_I - W y_S).
// mode 1 (product form, first half): y_I <- L^T y_I + W y_S.
template <typename T>
__global__ __launch_bounds__(WG) void k_elim_bwd(const ElimDesc* __restrict__ D, const T* __restrict__ arena,
                                                 const int32_t* __restrict__ slots, const int32_t* __restrict__ nslots,
                                                 T* __restrict__ y, int64_t ldy, int mode) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const ElimDesc d = D[blockIdx.x];
  const int m = d.m, k = d.k;
  T* ys = reinterpret_cast<T*>(smem_raw);
  T* g = ys + m;
  const int64_t R = (int64_t)m + k;
  const T* C = arena + d.front_off;
  T* yv = y + blockIdx.y * ldy;
  const int32_t* sl = slots + d.slot_off;
  const int32_t* ns = nslots + d.nslot_off;
  for (int i = threadIdx.x; i < m; i += WG) ys[i] = yv[sl[i]];
  for (int a = threadIdx.x; a < k; a += WG) g[a] = yv[ns[a]];
  __syncthreads();
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  if (mode == 0) {
    for (int j = w; j < m; j += WG / WAVE) {
      T acc = 0;
      for (int a = lane; a < k; a += WAVE) acc += C[(m + a) + (int64_t)j * R] * g[a];
      acc = wave_sum(acc);
      if (lane == 0) ys[j] -= acc;
    }
    __syncthreads();
    wg_trsv_lower_t(C, R, m, ys);
    for (int i = threadIdx.x; i < m; i += WG) yv[sl[i]] = ys[i];
  } else {
    // out_j = sum_{i >= j} L_ij ys_i + sum_a W^T_aj g_a
    T* out = g + k;
    for (int j = w; j < m; j += WG / WAVE) {
      T acc = 0;
      for (int i = j + lane; i < m; i += WAVE) acc += C[i + (int64_t)j * R] * ys[i];
      for (int a = lane; a < k; a += WAVE) acc += C[(m + a) + (int64_t)j * R] * g[a];
      acc = wave_sum(acc);
      if (lane == 0) out[j] = acc;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < m; i += WG) yv[sl[i]] = out[i];
  }
}

// Compressed separators: mode 0: y_B <- Q^T L^{-1} y_B; mode 1: y_B <- L^{-T} Q y_B;
// mode 2 (product): y_B <- Q^T L^T y_B; mode 3 (product): y_B <- L Q y_B.
template <typename T>
__global__ __launch_bounds__(WG) void k_comp_apply(const CompApply* __restrict__ A, const T* __restrict__ cf,
                                                   const T* __restrict__ nbuf, const T* __restrict__ tau_all,
                                                   const int32_t* __restrict__ slots, T* __restrict__ y, int64_t ldy,
                                                   int mode) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ T red[WG / WAVE];
  const CompApply a = A[blockIdx.x];
  const int s = a.s;
  T* ys = reinterpret_cast<T*>(smem_raw);
  T* tmp = ys + s;
  const T* L = cf + a.cf_off;
  const T* V = nbuf + a.v_off;
  const T* tau = tau_all + a.tau_off;
  T* yv = y + blockIdx.y * ldy;
  const int32_t* sl = slots + a.slot_off;
  for (int i = threadIdx.x; i < s; i += WG) ys[i] = yv[sl[i]];
  __syncthreads();
  auto qt = [&](bool transpose_order) {
    for (int kk = 0; kk < a.r; ++kk) {
      const int k = transpose_order ? kk : a.r - 1 - kk;
      T part = 0;
      for (int i = k + threadIdx.x; i < s; i += WG) part += (i == k ? T(1) : V[i + (int64_t)k * s]) * ys[i];
      const T wk = block_sum(part, red) * tau[k];
      for (int i = k + threadIdx.x; i < s; i += WG) ys[i] -= wk * (i == k ? T(1) : V[i + (int64_t)k * s]);
      __syncthreads();
    }
  };
  if (mode == 0) {
    wg_trsv_lower(L, a.ld, s, ys);
    qt(true);
  } else if (mode == 1) {
    qt(false);
    wg_trsv_lower_t(L, a.ld, s, ys);
  } else if (mode == 2) {
    for (int j = threadIdx.x; j < s; j += WG) {
      T acc = 0;
      for (int i = j; i < s; ++i) acc += L[i + (int64_t)j * a.ld] * ys[i];
      tmp[j] = acc;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < s; i += WG) ys[i] = tmp[i];
    __syncthreads();
    qt(true);
  } else {
    qt(false);
    for (int i = threadIdx.x; i < s; i += WG) {
      T acc = 0;
      for (int j = 0; j <= i; ++j) acc += L[i + (int64_t)j * a.ld] * ys[j];
      tmp[i] = acc;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < s; i += WG) ys[i] = tmp[i];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < s; i += WG) yv[sl[i]] = ys[i];
}

// ---------------------------------------------------------------------------
// Bandwidth-oriented apply sweeps (Sec. 4.7).  The factor panel of an
// interior, [L ; W^T] ((m+k) x m, column major), is read exactly once per
// sweep with coalesced column accesses; 64 x 64 diagonal triangles are staged
// in LDS (padded ld, conflict-free for L and L^T access) and solved by one
// wave, everything below them is a GEMV with all 256 threads.
// ---------------------------------------------------------------------------

constexpr int DB = 64;
constexpr int DLD = DB + 1;

// Lower triangle of the diagonal block [jb, jb + nb) of C into D, with the
// reciprocal of the diagonal stored on the diagonal; entries more than bw
// below the diagonal are known zeros and not read.  Every load of a round
// (U per thread) is issued before its stores.
template <typename T, int U = 8>
__device__ __forceinline__ void stage_diag(const T* __restrict__ C, int64_t ld, int jb, int nb, T* D, int bw) {
  const int n = nb * nb;
  for (int base = 0; base < n; base += U * WG) {
    T t[U];
    int ii[U], jj[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = base + u * WG + (int)threadIdx.x;
      ii[u] = idx % nb;
      jj[u] = idx < n ? idx / nb : -1;
      const int i = ii[u], j = jj[u];
      t[u] = (j >= 0 && i >= j && i - j <= bw) ? C[(jb + i) + (int64_t)(jb + j) * ld] : T(0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (jj[u] >= 0) D[ii[u] + jj[u] * DLD] = (ii[u] == jj[u]) ? T(1) / t[u] : t[u];
  }
}

// Right-hand sides per workgroup in the apply kernels: the factor is read
// once for up to RCM columns (grid.y = ceil(nrhs / rc)).
constexpr int RCM = 4;

// Forward sweep of one interior: y_I <- L^{-1} y_I, t <- W^T y_I, for rc
// right-hand sides (columns blockIdx.y * rc ...) at once: the triangular
// chains of the columns run on different wavefronts, the block products
// share each factor load.
template <typename T, int RC>
__global__ __launch_bounds__(WG) void k_apply_fwd(const ElimDesc* __restrict__ D, const T* __restrict__ arena,
                                                  const int32_t* __restrict__ slots, T* __restrict__ y, int64_t ldy,
                                                  T* __restrict__ tscr, int64_t ldt, int nrhs) {
  constexpr int rc = RC;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* Dg = reinterpret_cast<T*>(smem_raw);
  T* v = Dg + DB * DLD;
  const ElimDesc d = D[blockIdx.x];
  const int m = d.m, k = d.k, R = m + k, Rp = (R + 3) & ~3;
  const int c0 = blockIdx.y * rc, nc = min(rc, nrhs - c0);
  const T* C = arena + d.front_off;
  const int32_t* sl = slots + d.slot_off;
  for (int idx = threadIdx.x; idx < R * nc; idx += WG) {
    const int i = idx % R, c = idx / R;
    v[i + c * Rp] = i < m ? y[(int64_t)(c0 + c) * ldy + sl[i]] : T(0);
  }
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  for (int jb = 0; jb < m; jb += DB) {
    const int nb = min(DB, m - jb);
    stage_diag(C, R, jb, nb, Dg, d.bw);
    __syncthreads();
    if (w < nc) {
      // lane j finishes x_j at step j (scaled by its reciprocal pivot) and
      // the value is broadcast through a scalar register
      T* vc = v + w * Rp;
      T x = lane < nb ? vc[jb + lane] : T(0);
      const T dinv = lane < nb ? Dg[lane + lane * DLD] : T(0);
      for (int j = 0; j < nb; ++j) {
        const T xj = lane_bcast(x * dinv, j);
        if (lane == j) x = xj;
        else if (lane > j) x -= Dg[lane + j * DLD] * xj;
      }
      if (lane < nb) vc[jb + lane] = x;
    }
    __syncthreads();
    // rows below the block: the band rows of L_I and all rows of W^T
    const int band = min(m, jb + nb + d.bw) - (jb + nb);
    for (int ii = threadIdx.x; ii < band + k; ii += WG) {
      const int i = ii < band ? jb + nb + ii : m + (ii - band);
      const T* ci = C + i + (int64_t)jb * R;
      T acc[RC];
#pragma unroll
      for (int c = 0; c < RC; ++c) acc[c] = 0;
#pragma unroll 16
      for (int j = 0; j < nb; ++j) {
        const T cij = ci[(int64_t)j * R];
#pragma unroll
        for (int c = 0; c < RC; ++c) acc[c] += cij * v[jb + j + c * Rp];
      }
#pragma unroll
      for (int c = 0; c < RC; ++c)
        if (c < nc) v[i + c * Rp] -= acc[c];
    }
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < R * nc; idx += WG) {
    const int i = idx % R, c = idx / R;
    if (i < m) y[(int64_t)(c0 + c) * ldy + sl[i]] = v[i + c * Rp];
    else tscr[(int64_t)(c0 + c) * ldt + d.t_off + (i - m)] = -v[i + c * Rp];
  }
}

// Backward sweep of one interior: y_I <- L^{-T} (y_I - W y_S), rc columns.
template <typename T, int RC>
__global__ __launch_bounds__(WG) void k_apply_bwd(const ElimDesc* __restrict__ D, const T* __restrict__ arena,
                                                  const int32_t* __restrict__ slots,
                                                  const int32_t* __restrict__ nslots, T* __restrict__ y,
                                                  int64_t ldy, int nrhs) {
  constexpr int rc = RC;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* Dg = reinterpret_cast<T*>(smem_raw);
  T* v = Dg + DB * DLD;
  const ElimDesc d = D[blockIdx.x];
  const int m = d.m, k = d.k, R = m + k, Rp = (R + 3) & ~3;
  const int c0 = blockIdx.y * rc, nc = min(rc, nrhs - c0);
  const T* C = arena + d.front_off;
  const int32_t* sl = slots + d.slot_off;
  const int32_t* ns = nslots + d.nslot_off;
  for (int idx = threadIdx.x; idx < R * nc; idx += WG) {
    const int i = idx % R, c = idx / R;
    v[i + c * Rp] = y[(int64_t)(c0 + c) * ldy + (i < m ? sl[i] : ns[i - m])];
  }
  __syncthreads();
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  for (int bj = (m + DB - 1) / DB - 1; bj >= 0; --bj) {
    const int jb = bj * DB, nb = min(DB, m - jb), below = jb + nb;
    const int band = min(m, below + d.bw) - below;   // band rows of L_I below the block, then W^T
    // two columns per pass so that their loads and reductions overlap
    for (int j = 2 * w; j < nb; j += 2 * (WG / WAVE)) {
      const bool two = j + 1 < nb;
      const T* cj = C + (int64_t)(jb + j) * R;
      const T* ck = cj + R;
      T a0[RC], a1[RC];
#pragma unroll
      for (int c = 0; c < RC; ++c) a0[c] = a1[c] = 0;
#pragma unroll 4
      for (int ii = lane; ii < band + k; ii += WAVE) {
        const int i = ii < band ? below + ii : m + (ii - band);
        const T c0v = cj[i], c1v = two ? ck[i] : T(0);
#pragma unroll
        for (int c = 0; c < RC; ++c) {
          const T vi = v[i + c * Rp];
          a0[c] += c0v * vi;
          a1[c] += c1v * vi;
        }
      }
#pragma unroll
      for (int c = 0; c < RC; ++c)
        if (c < nc) {
          const T s0 = wave_sum(a0[c]), s1 = wave_sum(a1[c]);
          if (lane == 0) {
            v[jb + j + c * Rp] -= s0;
            if (two) v[jb + j + 1 + c * Rp] -= s1;
          }
        }
    }
    stage_diag(C, R, jb, nb, Dg, d.bw);
    __syncthreads();
    if (w < nc) {
      T* vc = v + w * Rp;
      T x = lane < nb ? vc[jb + lane] : T(0);
      const T dinv = lane < nb ? Dg[lane + lane * DLD] : T(0);
      for (int j = nb - 1; j >= 0; --j) {
        const T xj = lane_bcast(x * dinv, j);
        if (lane == j) x = xj;
        else if (lane < j) x -= Dg[j + lane * DLD] * xj;
      }
      if (lane < nb) vc[jb + lane] = x;
    }
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < m * nc; idx += WG) {
    const int i = idx % m, c = idx / m;
    y[(int64_t)(c0 + c) * ldy + sl[i]] = v[i + c * Rp];
  }
}

// ---------------------------------------------------------------------------
// One right-hand side on a level whose interiors have at most 64 unknowns
// (the upper levels of a 2D grid): one workgroup per front.  Every load of
// the front is issued before any wait (the triangle of L_I masked to its
// band, L_SI, the slots, then y; buffer loads, out-of-range ones read 0), so
// a front waits for memory about twice; wavefront 0 then solves with the
// triangle in an LDS tile (row l of the tile holds the coefficients of row l's
// update, zero elsewhere: a row step is one read at a constant offset, a
// multiply, a readlane and a multiply-add, as in k_band1_solve), and the
// L_SI products run on all threads from LDS.
//   forward:  x = L_I^{-1} y_I, t = L_SI x (into the apply scratch);
//   backward: x = L_I^{-T} (y_I - L_SI^T y_S).
// The products are summed in the order of the sweeps that several columns
// take on the level (order 1: the banded sweeps, four partial sums over the
// residue classes of the summation index mod 4, added in class order; 0: the
// blocked sweeps, forward one running sum, backward lane-strided partial
// sums reduced by wave_sum), and the solve takes their steps, so a column
// gets the same values whatever the column count (a zero product can only
// turn a -0 into +0).
// LDS: the 64 x 65 tile, 1 / L_ll, x, y_S (kmax) and L_SI (k | 1 per column).
// ---------------------------------------------------------------------------
__host__ __device__ inline int64_t apply1_lds_elems(int kmax) {
  return (int64_t)WAVE * (WAVE + 1) + 2 * WAVE + kmax + (int64_t)(kmax | 1) * WAVE;
}

template <typename T, bool FWD>
__global__ __launch_bounds__(WG) void k_apply1(const ElimDesc* __restrict__ D, const T* __restrict__ arena,
                                               const int32_t* __restrict__ slots,
                                               const int32_t* __restrict__ nslots, T* __restrict__ y,
                                               T* __restrict__ tscr, int kmax, int order) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int E = sizeof(T), TL = WAVE + 1, U = 8;
  T* Tt = reinterpret_cast<T*>(smem_raw);   // 64 x TL
  T* dv = Tt + WAVE * TL;                    // 1 / L_ll (0 past m)
  T* xs = dv + WAVE;                         // x
  T* ys = xs + WAVE;                         // y_S (backward)
  T* Wl = ys + kmax;                         // L_SI(r, j) at Wl[r + j * KP]
  const ElimDesc d = D[blockIdx.x];
  const int m = d.m, k = d.k, R = m + k, bw = min(d.bw, max(m - 1, 0)), KP = k | 1;
  const int tid = threadIdx.x, lane = tid % WAVE;
  const auto rc = buf_res(arena + d.front_off, (int64_t)R * R * E);
  // triangle tile: position (l, j) of the tile, lanes consecutive in the
  // front's row index so that the loads are coalesced
  T tv[WAVE * WAVE / WG];
#pragma unroll
  for (int u = 0; u < WAVE * WAVE / WG; ++u) {
    const int p = tid + u * WG, a = p % WAVE, b = p / WAVE;
    // forward: (l, j) = (a, b), L[l][j] for j < l; backward: (l, j) = (b, a), L[j][l] for j > l
    const int l = FWD ? a : b, j = FWD ? b : a;
    const int ri = FWD ? l : j, ci = FWD ? j : l;   // L[ri][ci], ri > ci
    tv[u] = buf_ld(rc, buf_off(ri > ci && ri < m && ri - ci <= bw, ri + (int64_t)ci * R, E), T());
  }
  const T piv = buf_ld(rc, buf_off(tid < m, tid + (int64_t)tid * R, E), T());
  // L_SI, issued in rounds of U per thread before their stores
  const int nw = k * m;
  for (int base = 0; base < nw; base += U * WG) {
    T wv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = base + u * WG + tid, r = idx % max(k, 1), j = idx / max(k, 1);
      wv[u] = buf_ld(rc, buf_off(idx < nw, m + r + (int64_t)j * R, E), T());
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = base + u * WG + tid, r = idx % max(k, 1), j = idx / max(k, 1);
      if (idx < nw) Wl[r + j * KP] = wv[u];
    }
  }
  // slots and y (indices clamped into the front; fronts without interior or
  // separator rows read none)
  const int32_t* sl = slots + d.slot_off;
  const int32_t si = m > 0 ? sl[min(tid, m - 1)] : 0;
  int32_t sn = 0;
  if (!FWD && k > 0) sn = nslots[d.nslot_off + min(tid, k - 1)];
  const T yi = m > 0 ? y[si] : T(0);
  T yn = T(0);
  if (!FWD && k > 0) yn = y[sn];
#pragma unroll
  for (int u = 0; u < WAVE * WAVE / WG; ++u) {
    const int p = tid + u * WG, a = p % WAVE, b = p / WAVE;
    const int l = FWD ? a : b, j = FWD ? b : a;
    Tt[l * TL + j] = tv[u];
  }
  if (tid < WAVE) {
    dv[tid] = tid < m ? T(1) / piv : T(0);
    xs[tid] = tid < m ? yi : T(0);
  }
  if (!FWD && tid < k) ys[tid] = yn;
  __syncthreads();
  if (!FWD) {
    // y_I - L_SI^T y_S, column j summed over the separator rows
    if (order == 1) {
      if (tid < m) {
        T p[4] = {0, 0, 0, 0};
        for (int r = 0; r < k; ++r) p[r & 3] += Wl[r + tid * KP] * ys[r];
        T sum = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) sum += p[q];
        xs[tid] = xs[tid] - sum;
      }
    } else {
      const int w = tid / WAVE;
      for (int j = w; j < m; j += WG / WAVE) {
        T a = 0;
        for (int r = lane; r < k; r += WAVE) a += Wl[r + j * KP] * ys[r];
        const T sum = wave_sum(a);
        if (lane == 0) xs[j] = xs[j] - sum;
      }
    }
    __syncthreads();
  }
  if (tid < WAVE) {
    T x = xs[lane];
    const T dinv = dv[lane];
    const int m8 = (m + 7) & ~7;
    if (FWD) {
      for (int j0 = 0; j0 < m8; j0 += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const T xj = lane_bcast(x * dinv, j0 + u);
          x = x - Tt[lane * TL + j0 + u] * xj;
        }
      }
    } else {
      for (int j0 = m8 - 8; j0 >= 0; j0 -= 8) {
#pragma unroll
        for (int u = 7; u >= 0; --u) {
          const T xj = lane_bcast(x * dinv, j0 + u);
          x = x - Tt[lane * TL + j0 + u] * xj;
        }
      }
    }
    x = x * dinv;
    xs[lane] = x;
    if (lane < m) y[si] = x;
  }
  if (FWD) {
    __syncthreads();
    // t = L_SI x: thread r sums row r over the interior columns
    for (int r = tid; r < k; r += WG) {
      T sum = 0;
      if (order == 1) {
        T p[4] = {0, 0, 0, 0};
        for (int j = 0; j < m; ++j) p[j & 3] += Wl[r + j * KP] * xs[j];
#pragma unroll
        for (int q = 0; q < 4; ++q) sum += p[q];
      } else {
        for (int j = 0; j < m; ++j) sum += Wl[r + j * KP] * xs[j];
      }
      tscr[d.t_off + r] = sum;
    }
  }
}

// ---------------------------------------------------------------------------
// Banded apply sweeps, for levels whose interiors have a narrow M_II (lower
// bandwidth bw <= BAND_MAX, e.g. the finest interiors of a grid numbered
// naturally).  Each workgroup stages the band of L_I once in LDS by
// diagonals, Bd[r * ld + i] = L[i, i - r] (the reciprocal pivot at r = 0),
// with a row stride that keeps the lanes of one step on distinct banks.  The
// triangular solve runs on one wavefront per right-hand side, one row per
// lane in chunks of 64: the value finished at a step reaches the other lanes
// through a scalar register, and the lanes within the band below (above) it
// update.  The products with the L_SI rows of the panel use all 256 threads
// with coalesced column loads and sum in a fixed order.
// ---------------------------------------------------------------------------
constexpr int BAND_MAX = 64;

template <typename T>
__device__ __forceinline__ void stage_band(const T* __restrict__ C, int R, int m, int bw, T* Bd, int ld) {
  const int nb1 = bw + 1;
  for (int idx = threadIdx.x; idx < m * nb1; idx += WG) {
    const int j = idx / nb1, r = idx - j * nb1, i = j + r;
    if (i < m) {
      const T c = C[i + (int64_t)j * R];
      Bd[r * ld + i] = r == 0 ? T(1) / c : c;
    }
  }
}

// Workgroup gather from global memory into LDS, element idx from
// src[f(idx).x] to dst[f(idx).y], with every load of a round issued before
// its stores, so that a thread keeps U loads in flight instead of one.
template <typename T, int U, typename F>
__device__ __forceinline__ void lds_gather(T* dst, const T* __restrict__ src, int n, F f) {
  for (int base = 0; base < n; base += U * WG) {
    T t[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = base + u * WG + (int)threadIdx.x;
      if (idx < n) t[u] = src[f(idx).x];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = base + u * WG + (int)threadIdx.x;
      if (idx < n) dst[f(idx).y] = t[u];
    }
  }
}

// LDS elements of the banded sweeps for fronts up to (m, k, bw), RC columns.
__host__ __device__ constexpr int band_fwd_ld(int m) { return (m + 1) & ~1; }
__host__ __device__ constexpr int band_bwd_ld(int m) { return m | 1; }
__host__ __device__ inline int64_t band_fwd_lds(int m, int k, int bw, int rc) {
  (void)k;
  return (int64_t)(bw + 1) * band_fwd_ld(m) + (int64_t)rc * band_fwd_ld(m) + (int64_t)(WG / WAVE) * rc * WAVE;
}
__host__ __device__ inline int64_t band_bwd_lds(int m, int k, int bw, int rc, int tj) {
  const int64_t a = (int64_t)(bw + 1) * band_bwd_ld(m), b = (int64_t)tj * (k | 1);
  return (a > b ? a : b) + (int64_t)rc * band_bwd_ld(m) + (int64_t)rc * k + (int64_t)(WG / WAVE) * rc * WAVE;
}

// Forward sweep: y_I <- L_I^{-1} y_I and t = L_SI y_I (into the apply scratch).
// PK: the factor is read from its packed copy (contiguous, aligned) instead
// of the front.
template <typename T, int RC, bool PK>
__global__ __launch_bounds__(WG) void k_band_fwd(const ElimDesc* __restrict__ D, const T* __restrict__ arena,
                                                 const int32_t* __restrict__ slots, T* __restrict__ y, int64_t ldy,
                                                 T* __restrict__ tscr, int64_t ldt, int nrhs,
                                                 const T* __restrict__ pk) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const ElimDesc d = D[blockIdx.x];
  const int m = d.m, k = d.k, R = m + k, bw = min(d.bw, max(m - 1, 0));
  const int ld = band_fwd_ld(m);
  T* Bd = reinterpret_cast<T*>(smem_raw);
  T* v = Bd + (bw + 1) * ld;
  T* part = v + RC * ld;
  const int c0 = blockIdx.y * RC, nc = min(RC, nrhs - c0);
  const T* C = arena + d.front_off;
  const int32_t* sl = slots + d.slot_off;
  const T* PB = PK ? pk + d.pk_off : nullptr;
  const T* PL = PK ? PB + band_pk_lsi(m, bw) : nullptr;
  for (int idx = threadIdx.x; idx < m * nc; idx += WG) {
    const int i = idx % m, c = idx / m;
    v[c * ld + i] = y[(int64_t)(c0 + c) * ldy + sl[i]];
  }
  if (PK) {
    for (int idx = threadIdx.x; idx < (bw + 1) * ld; idx += WG) Bd[idx] = PB[idx];   // same layout
  } else {
    stage_band(C, R, m, bw, Bd, ld);
  }
  __syncthreads();
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  // rows i0 .. i0 + 63 of x = L_I^{-1} x by one wavefront (earlier rows final)
  auto solve_chunk = [&](T* vc, int i0) {
    const int i = i0 + lane, cn = min(WAVE, m - i0);
    const bool on = i < m;
    T x = on ? vc[i] : T(0);
    const T dinv = on ? Bd[i] : T(0);
    const int ic = min(i, m - 1);
    // columns of earlier chunks inside the band (their values are final),
    // ascending r; branch-free (clamped addresses, selected updates) so the
    // LDS reads do not wait on the chain
#pragma unroll 4
    for (int r = 1; r <= bw; ++r) {
      const T a = Bd[r * ld + ic], xv = vc[max(i - r, 0)];
      x = (r > lane && on && i - r >= 0) ? x - a * xv : x;
    }
    // steps past the chunk (cn up to a multiple of 8) broadcast zeros from
    // rows past m and change nothing
    const int cn8 = (cn + 7) & ~7;
    for (int j0 = 0; j0 < cn8; j0 += 8) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int jj = j0 + u, r = lane - jj;
        const T xj = lane_bcast(x * dinv, jj);
        const T a = Bd[min(max(r, 0), bw) * ld + ic];
        x = r == 0 ? xj : ((r > 0 && r <= bw && on) ? x - a * xj : x);
      }
    }
    if (on) vc[i] = x;
  };
  if (nc == 1 && k <= WAVE) {
    // one right-hand side, at most 64 separator rows: wavefront 0 solves the
    // chunks of 64 rows in turn while wavefronts 1-3 accumulate L_SI x over
    // the chunk finished before.  The partial sums are those of the general
    // path below (columns j = q mod 4 in ascending j, q = 0..3; wavefront 3
    // keeps q = 2 and 3) combined in the same order, so the result is the
    // same bits.
    const T* cr = PK ? PL + lane : C + m + lane;
    const int64_t cs = PK ? k : R;
    const int qa = w - 1, qb = w == 3 ? 3 : -1;
    T acca = T(0), accb = T(0);
    const int nch = (m + WAVE - 1) / WAVE;
    for (int ch = 0; ch <= nch; ++ch) {
      if (w == 0) {
        if (ch < nch) solve_chunk(v, ch * WAVE);
      } else if (ch > 0 && lane < k) {
        const int j0 = (ch - 1) * WAVE, j1 = min(m, j0 + WAVE);
#pragma unroll 4
        for (int j = j0 + qa; j < j1; j += 4) acca += cr[(int64_t)j * cs] * v[j];
        if (qb >= 0) {
#pragma unroll 4
          for (int j = j0 + qb; j < j1; j += 4) accb += cr[(int64_t)j * cs] * v[j];
        }
      }
      __syncthreads();
    }
    if (w > 0) {
      part[(qa * RC) * WAVE + lane] = acca;
      if (qb >= 0) part[(qb * RC) * WAVE + lane] = accb;
    }
    __syncthreads();
    if (w == 0 && lane < k) {
      T sum = 0;
      for (int q = 0; q < WG / WAVE; ++q) sum += part[(q * RC) * WAVE + lane];
      tscr[(int64_t)c0 * ldt + d.t_off + lane] = sum;
    }
    for (int idx = threadIdx.x; idx < m; idx += WG) y[(int64_t)c0 * ldy + sl[idx]] = v[idx];
    return;
  }
  if (w < nc) {
    T* vc = v + w * ld;
    for (int i0 = 0; i0 < m; i0 += WAVE) solve_chunk(vc, i0);
  }
  __syncthreads();
  // t = L_SI x: 64 rows per pass, the columns dealt to the wavefronts in turn
  for (int rb = 0; rb < k; rb += WAVE) {
    const int r = rb + lane;
    T acc[RC];
#pragma unroll
    for (int c = 0; c < RC; ++c) acc[c] = 0;
    if (r < k) {
      const T* cr = PK ? PL + r : C + m + r;
      const int64_t cs = PK ? k : R;
#pragma unroll 8
      for (int j = w; j < m; j += WG / WAVE) {
        const T cij = cr[(int64_t)j * cs];
#pragma unroll
        for (int c = 0; c < RC; ++c) acc[c] += cij * v[c * ld + j];
      }
    }
#pragma unroll
    for (int c = 0; c < RC; ++c) part[(w * RC + c) * WAVE + lane] = acc[c];
    __syncthreads();
    for (int idx = threadIdx.x; idx < WAVE * nc; idx += WG) {
      const int l = idx % WAVE, c = idx / WAVE;
      if (rb + l < k) {
        T sum = 0;
        for (int q = 0; q < WG / WAVE; ++q) sum += part[(q * RC + c) * WAVE + l];
        tscr[(int64_t)(c0 + c) * ldt + d.t_off + rb + l] = sum;
      }
    }
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < m * nc; idx += WG) {
    const int i = idx % m, c = idx / m;
    y[(int64_t)(c0 + c) * ldy + sl[i]] = v[c * ld + i];
  }
}

// Backward sweep: y_I <- L_I^{-T} (y_I - L_SI^T y_S).  The L_SI^T product
// stages tiles of tj <= 64 columns of the panel's L_SI rows transposed in
// LDS (the space the band takes afterwards), so each lane sums down one
// column, the rows dealt to the wavefronts in turn.
template <typename T, int RC, bool PK>
__global__ __launch_bounds__(WG) void k_band_bwd(const ElimDesc* __restrict__ D, const T* __restrict__ arena,
                                                 const int32_t* __restrict__ slots,
                                                 const int32_t* __restrict__ nslots, T* __restrict__ y,
                                                 int64_t ldy, int nrhs, int tj, const T* __restrict__ pk) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const ElimDesc d = D[blockIdx.x];
  const int m = d.m, k = d.k, R = m + k, bw = min(d.bw, max(m - 1, 0));
  const int ld = band_bwd_ld(m), ldk = k | 1;
  const int64_t big = max((int64_t)(bw + 1) * ld, (int64_t)tj * ldk);
  T* Bd = reinterpret_cast<T*>(smem_raw);   // the transposed tiles first, then the band
  T* v = Bd + big;
  T* ys = v + RC * ld;
  T* part = ys + RC * k;
  const int c0 = blockIdx.y * RC, nc = min(RC, nrhs - c0);
  const T* C = arena + d.front_off;
  const int32_t* sl = slots + d.slot_off;
  const int32_t* ns = nslots + d.nslot_off;
  for (int idx = threadIdx.x; idx < m * nc; idx += WG) {
    const int i = idx % m, c = idx / m;
    v[c * ld + i] = y[(int64_t)(c0 + c) * ldy + sl[i]];
  }
  for (int idx = threadIdx.x; idx < k * nc; idx += WG) {
    const int r = idx % k, c = idx / k;
    ys[c * k + r] = y[(int64_t)(c0 + c) * ldy + ns[r]];
  }
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const T* PB = PK ? pk + d.pk_off : nullptr;
  const T* PL = PK ? PB + band_pk_lsi(m, bw) : nullptr;
  for (int j0 = 0; j0 < m; j0 += tj) {
    const int cw = min(tj, m - j0);
    if (PK) {
      const T* src = PL + (int64_t)j0 * k;
      lds_gather<T, 8>(Bd, src, k * cw, [=](int idx) { return make_int2(idx, (idx / k) * ldk + idx % k); });
    } else {
      for (int idx = threadIdx.x; idx < k * cw; idx += WG) {
        const int r = idx % k, jl = idx / k;
        Bd[jl * ldk + r] = C[m + r + (int64_t)(j0 + jl) * R];
      }
    }
    __syncthreads();
    T acc[RC];
#pragma unroll
    for (int c = 0; c < RC; ++c) acc[c] = 0;
    if (lane < cw)
      for (int r = w; r < k; r += WG / WAVE) {
        const T wr = Bd[lane * ldk + r];
#pragma unroll
        for (int c = 0; c < RC; ++c) acc[c] += wr * ys[c * k + r];
      }
#pragma unroll
    for (int c = 0; c < RC; ++c) part[(w * RC + c) * WAVE + lane] = acc[c];
    __syncthreads();
    for (int idx = threadIdx.x; idx < WAVE * nc; idx += WG) {
      const int l = idx % WAVE, c = idx / WAVE;
      if (l < cw) {
        T sum = 0;
        for (int q = 0; q < WG / WAVE; ++q) sum += part[(q * RC + c) * WAVE + l];
        v[c * ld + j0 + l] -= sum;
      }
    }
    __syncthreads();
  }
  if (PK) {
    const int pld = band_pk_ld(m);
    lds_gather<T, 8>(Bd, PB, (bw + 1) * m, [=](int idx) {
      const int r = idx / m, i = idx - r * m;
      return make_int2(r * pld + i, r * ld + i);
    });
  } else {
    stage_band(C, R, m, bw, Bd, ld);
  }
  __syncthreads();
  if (w < nc) {
    T* vc = v + w * ld;
    for (int i0 = ((m - 1) / WAVE) * WAVE; i0 >= 0; i0 -= WAVE) {
      const int i = i0 + lane, cn = min(WAVE, m - i0);
      const bool on = i < m;
      T x = on ? vc[i] : T(0);
      const T dinv = on ? Bd[i] : T(0);
      // rows of later chunks inside the band (their values are final),
      // ascending r; branch-free as in the forward sweep
#pragma unroll 4
      for (int r = 1; r <= bw; ++r) {
        const int ir = min(i + r, m - 1);
        const T a = Bd[r * ld + ir], xv = vc[ir];
        x = (r >= WAVE - lane && on && i + r < m) ? x - a * xv : x;
      }
      const int cn8 = (cn + 7) & ~7;
      for (int j0 = cn8 - 8; j0 >= 0; j0 -= 8) {
#pragma unroll
        for (int u = 7; u >= 0; --u) {
          const int jj = j0 + u, r = jj - lane;
          const T xj = lane_bcast(x * dinv, jj);
          const T a = Bd[min(max(r, 0), bw) * ld + min(i0 + jj, m - 1)];
          x = r == 0 ? xj : ((r > 0 && r <= bw && jj < cn) ? x - a * xj : x);
        }
      }
      if (on) vc[i] = x;
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < m * nc; idx += WG) {
    const int i = idx % m, c = idx / m;
    y[(int64_t)(c0 + c) * ldy + sl[i]] = v[c * ld + i];
  }
}

// T_B = Q^T L_B^{-1} (s x s) for every compressed separator, so that each
// apply of B is one dense matrix-vector product (forward) or its transpose.
// Columns are independent: workgroup blockIdx.y forms columns
// [CEB * blockIdx.y, CEB * (blockIdx.y + 1)) of T_B.
constexpr int CEB = 64;
// ---------------------------------------------------------------------------
// Banded interior sweeps with one right-hand side, split by what bounds
// them (the level-1 interiors of a grid: lower bandwidth bw < 32, at most 64
// separator rows, packed factor copy):
//  * the band solves x = L_I^{-1} y_I and x = L_I^{-T} y_I are a chain of m
//    dependent row steps over few bytes (the band): one wavefront per front,
//    one 64-row chunk at a time, x and the band of every chunk in registers;
//  * the products with L_SI (t = L_SI x forward, y_I - L_SI^T y_S backward)
//    stream most of the factor's bytes: four wavefronts per front, each over
//    one residue class of the summation index, combined in LDS.
// The products, partial sums and their order are those of k_band_fwd /
// k_band_bwd, so the same values (see k_band1_solve for the sign of zeros).
// ---------------------------------------------------------------------------
constexpr int B1_FRONTS = WG / WAVE;
__host__ __device__ inline int band1_xs(int mmax) { return (mmax + WAVE - 1) / WAVE * WAVE; }
// fronts of at most B1_MAXC 64-row chunks: the band of all of them is loaded
// into registers at once
constexpr int B1_MAXC = 4;
// LDS of a band solve (per wavefront): S, 64 rows of band1_ls(NB) (the
// entries of a row that one group of eight steps can reach), E, NB rows of
// band1_le(NB) (the entries that reach into the neighbouring chunk), and 64
// zeros.  Odd row lengths, so that 64 lanes reading one entry of their own
// row each hit distinct banks.
__host__ __device__ constexpr int band1_ls(int nb) { return (nb + 13) | 1; }
__host__ __device__ constexpr int band1_le(int nb) { return nb | 1; }
__host__ __device__ inline int64_t band1_lds_elems(int mmax, int nb) {
  (void)mmax;
  return (int64_t)WAVE * band1_ls(nb) + (int64_t)nb * band1_le(nb) + WAVE;
}

// x = L_I^{-1} y_I (forward) or x = L_I^{-T} y_I (backward) for the fronts
// list[0..n), one per wavefront (blockDim.x / 64 per workgroup), y in slot
// order.  NB >= bw + 1 (17 or 32), m <= 64 * B1_MAXC.
//
// Lane l owns row i = i0 + l of the 64-row chunk at i0 and keeps x_i in a
// register.  The chunk is solved in row steps j = 0..63 (backward 63..0):
// x_j / L_jj is broadcast from lane j (readlane) and every lane subtracts its
// coefficient of x_j times it, zero for the rows the step does not touch.
// The steps go in groups of eight; the lanes a group touches read their
// coefficients from their row of S at eight consecutive offsets (the row
// holds the band entries of row i, forward, or of column i, backward, at
// their distance from the diagonal, zeros around them), the others from the
// zero block, so a step is a read at a constant offset, one multiply, one
// readlane and one multiply-add.  The entries reaching into the neighbouring
// chunk (already solved) are applied first from E, with the neighbour's
// final values broadcast from its registers.  Positions of S and E written
// for one chunk are the same for every chunk (entries past bw or m written
// as zeros), so both are cleared once.  A lane's own step and the steps after
// it add zero products and its result is x_i / L_ii at the end; the touched
// steps are those of k_band_fwd / k_band_bwd in the same order, so the same
// values (a zero product can turn a -0 into +0).  The band of every chunk,
// the slots and y are loaded first, all issued unconditionally (indices
// clamped into the front), so that a front waits for global memory about
// twice.
template <typename T, int NB, bool FWD>
__global__ __launch_bounds__(WG) void k_band1_solve(const ElimDesc* __restrict__ D, const int32_t* __restrict__ list,
                                                    int n, const int32_t* __restrict__ slots, T* __restrict__ y,
                                                    const T* __restrict__ pk, int lds_per_wave) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int LS = band1_ls(NB), LE = band1_le(NB);
  // S offset of a touched row at the first step of a group: forward, the
  // entry L[i][i - r] sits at OFF - r; backward, L[i + r][i] at OFF + r
  constexpr int OFF = FWD ? NB + 6 : 6;
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int fi = blockIdx.x * (blockDim.x / WAVE) + w;   // one front per wavefront
  if (fi >= n) return;   // whole wavefront: no workgroup barrier below
  const ElimDesc d = D[list[fi]];
  const int m = d.m, bw = min(d.bw, max(m - 1, 0));
  const int pld = band_pk_ld(m);
  T* S = reinterpret_cast<T*>(smem_raw) + (int64_t)w * lds_per_wave;
  T* E = S + WAVE * LS;
  T* Z = E + NB * LE;
  const int ZO = WAVE * LS + NB * LE;   // offset of the zeros from S
  const T* PB = pk + d.pk_off;
  const int32_t* sl = slots + d.slot_off;
  const int nch = (m + WAVE - 1) / WAVE;
  // band of every chunk, nbs[c][r] = PB[r][64 c + lane], then y
  T nbs[B1_MAXC][NB];
#pragma unroll
  for (int c = 0; c < B1_MAXC; ++c) {
    const int ic = min(c * WAVE + lane, m - 1);
#pragma unroll
    for (int r = 0; r < NB; ++r) nbs[c][r] = PB[(int64_t)min(r, bw) * pld + ic];
  }
  int32_t sv[B1_MAXC];
  T xr[B1_MAXC];
#pragma unroll
  for (int c = 0; c < B1_MAXC; ++c) sv[c] = sl[min(c * WAVE + lane, m - 1)];
#pragma unroll
  for (int c = 0; c < B1_MAXC; ++c) xr[c] = y[sv[c]];
#pragma unroll
  for (int p = 0; p < LS; ++p) S[lane * LS + p] = T(0);
  if (lane < NB)
    for (int p = 0; p < LE; ++p) E[lane * LE + p] = T(0);
  Z[lane] = T(0);
  __builtin_amdgcn_wave_barrier();
  auto chunk = [&](const int c, const T (&nb)[NB], T& xc, const T& xn) {
    // xn: the registers of the neighbouring chunk (solved before)
    const int i0 = c * WAVE, i = i0 + lane, cn = min(WAVE, m - i0);
    const bool on = i < m;
    T x = on ? xc : T(0);
    const int cn8 = (cn + 7) & ~7;   // steps past the chunk broadcast zeros from rows past m
    if (FWD) {
      // row i: L[i][i - r] = nb[r] into S at OFF - r; the entries with
      // i - r before the chunk (r > l) also into E[l][r - l]
#pragma unroll
      for (int r = 1; r < NB; ++r) {
        const T v = ((r <= bw) & on) ? nb[r] : T(0);
        S[lane * LS + OFF - r] = v;
        if (r > lane) E[lane * LE + r - lane] = c > 0 ? v : T(0);
      }
      __builtin_amdgcn_wave_barrier();
      // columns i0 - k of the earlier chunk inside the band (final values,
      // lane 64 - k of its registers), k = r - l ascending
      const int eb = lane < NB - 1 ? lane * LE : ZO - WAVE * LS;
#pragma unroll
      for (int k = 1; k < NB; ++k) x = x - E[eb + k] * lane_bcast(xn, WAVE - k);
      const T dinv = nb[0];
      for (int j0 = 0; j0 < cn8; j0 += 8) {
        const bool touched = (lane >= j0 + 1) & (lane <= j0 + 7 + bw);
        const int sb = touched ? lane * LS + j0 - lane + OFF : ZO;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const T xj = lane_bcast(x * dinv, j0 + u);
          x = x - S[sb + u] * xj;
        }
      }
      xc = x * dinv;
    } else {
      // rows i0 + 64 + k of the later chunk inside the band first (final
      // values, lane k of its registers), ascending k; their entries
      // L[i0 + 64 + k][i] were written to E by that chunk
      const int e0 = WAVE - (NB - 1);
      const int eb = lane >= e0 ? (lane - e0) * LE : ZO - WAVE * LS;
#pragma unroll
      for (int k = 0; k < NB - 1; ++k) x = x - E[eb + k] * lane_bcast(xn, k);
      __builtin_amdgcn_wave_barrier();
      // column i: L[i + r][i] = nb[r] into the S row of lane l - r at
      // OFF + r; for l < r (rows of the chunk before) into E[NB - 1 + l - r][l],
      // read by that chunk
#pragma unroll
      for (int r = 1; r < NB; ++r) {
        const T v = ((r <= bw) & on) ? nb[r] : T(0);
        const int row = lane - r;
        const int pos = row >= 0 ? row * LS + OFF + r : WAVE * LS + (NB - 1 + row) * LE + lane;
        S[pos] = v;
      }
      __builtin_amdgcn_wave_barrier();
      const T dinv = nb[0];
      for (int j0 = cn8 - 8; j0 >= 0; j0 -= 8) {
        const bool touched = (lane >= j0 - bw) & (lane <= j0 + 6);
        const int sb = touched ? lane * LS + j0 - lane + OFF : ZO;
#pragma unroll
        for (int u = 7; u >= 0; --u) {
          const T xj = lane_bcast(x * dinv, j0 + u);
          x = x - S[sb + u] * xj;
        }
      }
      xc = x * dinv;
    }
    __builtin_amdgcn_wave_barrier();
  };
  const T zero = T(0);
  if (FWD) {
#pragma unroll
    for (int c = 0; c < B1_MAXC; ++c)
      if (c < nch) chunk(c, nbs[c], xr[c], c > 0 ? xr[c > 0 ? c - 1 : 0] : zero);
  } else {
#pragma unroll
    for (int c = B1_MAXC - 1; c >= 0; --c)
      if (c < nch) chunk(c, nbs[c], xr[c], c + 1 < nch ? xr[c + 1 < B1_MAXC ? c + 1 : c] : zero);
  }
#pragma unroll
  for (int c = 0; c < B1_MAXC; ++c)
    if (c * WAVE + lane < m) y[sv[c]] = xr[c];
}

// t = L_SI x (forward): one workgroup per front; wavefront q sums the
// columns j = q mod 4 in ascending j for the separator row of its lane, and
// the four partial sums are added in the order q = 0..3.
template <typename T>
__global__ __launch_bounds__(WG) void k_band1_lsi(const ElimDesc* __restrict__ D, const int32_t* __restrict__ slots,
                                                  const T* __restrict__ y, T* __restrict__ tscr,
                                                  const T* __restrict__ pk, int xs_elems) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* xs = reinterpret_cast<T*>(smem_raw);   // x (m <= xs_elems)
  T* part = xs + xs_elems;                  // 4 x 64 partial sums
  const ElimDesc d = D[blockIdx.x];
  const int m = d.m, k = d.k, bw = min(d.bw, max(m - 1, 0));
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int32_t* sl = slots + d.slot_off;
  for (int i = threadIdx.x; i < m; i += WG) xs[i] = y[sl[i]];
  __syncthreads();
  T acc = 0;
  if (lane < k) {
    const T* cr = pk + d.pk_off + band_pk_lsi(m, bw) + lane;
#pragma unroll 16
    for (int j = w; j < m; j += 4) acc += cr[(int64_t)j * k] * xs[j];
  }
  part[w * WAVE + lane] = acc;
  __syncthreads();
  if (w == 0 && lane < k) {
    T sum = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) sum += part[q * WAVE + lane];
    tscr[d.t_off + lane] = sum;
  }
}

// y_I <- y_I - L_SI^T y_S (backward): one workgroup per front; 64-column
// tiles of L_SI staged in LDS so that the lane of column j reads its column;
// wavefront q sums the rows r = q mod 4 in ascending r, the partial sums are
// added in the order q = 0..3 and subtracted.
template <typename T>
__global__ __launch_bounds__(WG) void k_band1_lsit(const ElimDesc* __restrict__ D, const int32_t* __restrict__ slots,
                                                   const int32_t* __restrict__ nslots, T* __restrict__ y,
                                                   const T* __restrict__ pk) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const ElimDesc d = D[blockIdx.x];
  const int m = d.m, k = d.k, bw = min(d.bw, max(m - 1, 0));
  const int ldk = k | 1;
  T* tile = reinterpret_cast<T*>(smem_raw);   // WAVE columns x k rows, ld ldk
  T* ys = tile + WAVE * (BE_KMAX | 1);        // y_S (k)
  T* part = ys + BE_KMAX;                     // 4 x 64 partial sums
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int32_t* sl = slots + d.slot_off;
  const int32_t* ns = nslots + d.nslot_off;
  const T* PL = pk + d.pk_off + band_pk_lsi(m, bw);
  for (int r = threadIdx.x; r < k; r += WG) ys[r] = y[ns[r]];
  for (int j0 = 0; j0 < m; j0 += WAVE) {
    const int cw = min(WAVE, m - j0);
    lds_gather<T, 8>(tile, PL + (int64_t)j0 * k, k * cw,
                     [=](int idx) { return make_int2(idx, (idx / k) * ldk + idx % k); });
    __syncthreads();
    T acc = 0;
    if (lane < cw)
      for (int r = w; r < k; r += 4) acc += tile[lane * ldk + r] * ys[r];
    part[w * WAVE + lane] = acc;
    __syncthreads();
    if (w == 0 && lane < cw) {
      T sum = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) sum += part[q * WAVE + lane];
      y[sl[j0 + lane]] -= sum;
    }
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(WG) void k_comp_explicit(const CompApply* __restrict__ A, const T* __restrict__ cf,
                                                      const T* __restrict__ nbuf, const T* __restrict__ tau_all,
                                                      T* __restrict__ tb) {
  const CompApply a = A[blockIdx.x];
  const int s = a.s, c0 = blockIdx.y * CEB;
  if (c0 >= s) return;
  const int nc = min(CEB, s - c0);
  T* X = tb + a.t_off + (int64_t)c0 * s;
  for (int idx = threadIdx.x; idx < s * nc; idx += WG) X[idx] = (idx % s == c0 + idx / s) ? T(1) : T(0);
  __syncthreads();
  // rows above c0 of L_B^{-1} I[:, c0:] are zero: solve only the trailing system
  wg_trsm_lower(cf + a.cf_off + c0 + (int64_t)c0 * a.ld, a.ld, s - c0, X + c0, s, nc);
  wg_apply_qt(nbuf + a.v_off, s, tau_all + a.tau_off, s, a.r, X, s, nc);
}

// k_comp_apply_t for a separator of at most SB <= 64 rows: the entries of
// T_B each thread multiplies are loaded into registers before the first wait
// (mode 0: row i, by the threads of rows; mode 1: one entry of each of the
// wavefront's columns per lane), zero past s so that their products add
// zeros; the arithmetic is that of the general path.
template <typename T, int SB>
__device__ __forceinline__ void comp_apply_small(const T* __restrict__ X, const int32_t* __restrict__ sl,
                                                 T* __restrict__ y, int64_t ldy, int mode, int s, int c0, int nc,
                                                 T* ys, T* out) {
  constexpr int E = sizeof(T), NW = WG / WAVE, NQ = (SB + NW - 1) / NW;
  const auto rx = buf_res(X, (int64_t)s * s * E);
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  T xr[SB];
  if (mode == 0) {
    const int i = threadIdx.x;
    if (i < SB)
#pragma unroll
      for (int j = 0; j < SB; ++j) xr[j] = buf_ld(rx, buf_off(i < s && j < s, i + (int64_t)j * s, E), T());
  } else if (lane < SB) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int j = w + q * NW;
      xr[q] = buf_ld(rx, buf_off(lane < s && j < s, lane + (int64_t)j * s, E), T());
    }
  }
  for (int idx = threadIdx.x; idx < s * nc; idx += WG) {
    const int i = idx % s, c = idx / s;
    ys[i + c * s] = y[(int64_t)(c0 + c) * ldy + sl[i]];
  }
  __syncthreads();
  if (mode == 0) {
    const int i = threadIdx.x;
    if (i < s)
      for (int c = 0; c < nc; ++c) {
        T acc = 0;
#pragma unroll
        for (int j = 0; j < SB; ++j) acc += xr[j] * (j < s ? ys[j + c * s] : T(0));
        out[i + c * s] = acc;
      }
  } else {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int j = w + q * NW;
      if (j < s)
        for (int c = 0; c < nc; ++c) {
          T acc = 0;
          if (lane < s) acc += xr[q] * ys[lane + c * s];
          const T t = wave_sum(acc);
          if (lane == 0) out[j + c * s] = t;
        }
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < s * nc; idx += WG) {
    const int i = idx % s, c = idx / s;
    y[(int64_t)(c0 + c) * ldy + sl[i]] = out[i + c * s];
  }
}

// mode 0: y_B <- T_B y_B; mode 1: y_B <- T_B^T y_B; rc columns per workgroup.
// SB > 0: the level's separators have at most SB rows (comp_apply_small);
// 0: the general path only.
template <typename T, int SB>
__global__ __launch_bounds__(WG) void k_comp_apply_t(const CompApply* __restrict__ A, const T* __restrict__ tb,
                                                     const int32_t* __restrict__ slots, T* __restrict__ y,
                                                     int64_t ldy, int mode, int nrhs, int rc) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const CompApply a = A[blockIdx.x];
  const int s = a.s;
  const int c0 = blockIdx.y * rc, nc = min(rc, nrhs - c0);
  T* ys = reinterpret_cast<T*>(smem_raw);
  T* out = ys + s * rc;
  const T* X = tb + a.t_off;
  const int32_t* sl = slots + a.slot_off;
  if (SB > 0 && s <= SB) {
    comp_apply_small<T, (SB > 0 ? SB : 16)>(X, sl, y, ldy, mode, s, c0, nc, ys, out);
    return;
  }
  for (int idx = threadIdx.x; idx < s * nc; idx += WG) {
    const int i = idx % s, c = idx / s;
    ys[i + c * s] = y[(int64_t)(c0 + c) * ldy + sl[i]];
  }
  __syncthreads();
  if (mode == 0) {
    for (int i = threadIdx.x; i < s; i += WG) {
      T acc[RCM];
#pragma unroll
      for (int c = 0; c < RCM; ++c) acc[c] = 0;
#pragma unroll 8
      for (int j = 0; j < s; ++j) {
        const T xij = X[i + (int64_t)j * s];
#pragma unroll
        for (int c = 0; c < RCM; ++c)
          if (c < nc) acc[c] += xij * ys[j + c * s];
      }
#pragma unroll
      for (int c = 0; c < RCM; ++c)
        if (c < nc) out[i + c * s] = acc[c];
    }
  } else {
    const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
    for (int j = w; j < s; j += WG / WAVE) {
      T acc[RCM];
#pragma unroll
      for (int c = 0; c < RCM; ++c) acc[c] = 0;
#pragma unroll 4
      for (int i = lane; i < s; i += WAVE) {
        const T xij = X[i + (int64_t)j * s];
#pragma unroll
        for (int c = 0; c < RCM; ++c)
          if (c < nc) acc[c] += xij * ys[i + c * s];
      }
#pragma unroll
      for (int c = 0; c < RCM; ++c)
        if (c < nc) {
          const T t = wave_sum(acc[c]);
          if (lane == 0) out[j + c * s] = t;
        }
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < s * nc; idx += WG) {
    const int i = idx % s, c = idx / s;
    y[(int64_t)(c0 + c) * ldy + sl[i]] = out[i + c * s];
  }
}

// Large separators: mode 0 out = T_B y_B (64 rows per workgroup, columns split
// over the wavefronts), mode 1 out = T_B^T y_B (64 columns per workgroup, one
// wavefront per column), rc right-hand sides; out goes to cw (ld ldc) and
// k_comp_scatter moves it into y, so no workgroup overwrites an input another
// one still reads.
template <typename T>
__global__ __launch_bounds__(WG) void k_comp_apply_big(const CompApply* __restrict__ A, const T* __restrict__ tb,
                                                       const int32_t* __restrict__ slots, const T* __restrict__ y,
                                                       int64_t ldy, int mode, int nrhs, int rc, T* __restrict__ cw,
                                                       int64_t ldc) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const CompApply a = A[blockIdx.x];
  const int s = a.s, sp = (s + 3) & ~3, b0 = blockIdx.y * 64;
  if (b0 >= s) return;
  const int q0 = blockIdx.z * rc, nc = min(rc, nrhs - q0);
  T* ys = reinterpret_cast<T*>(smem_raw);
  T* part = ys + sp * rc;
  const T* X = tb + a.t_off;
  const int32_t* sl = slots + a.slot_off;
  for (int idx = threadIdx.x; idx < s * nc; idx += WG) {
    const int i = idx % s, q = idx / s;
    ys[i + q * sp] = y[(int64_t)(q0 + q) * ldy + sl[i]];
  }
  __syncthreads();
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  if (mode == 0) {
    const int i = b0 + lane;
    T acc[RCM];
#pragma unroll
    for (int q = 0; q < RCM; ++q) acc[q] = 0;
    if (i < s)
      for (int j = w; j < s; j += WG / WAVE) {
        const T x = X[i + (int64_t)j * s];
#pragma unroll
        for (int q = 0; q < RCM; ++q)
          if (q < nc) acc[q] += x * ys[j + q * sp];
      }
#pragma unroll
    for (int q = 0; q < RCM; ++q)
      if (q < nc) part[(q * (WG / WAVE) + w) * WAVE + lane] = acc[q];
    __syncthreads();
    if (w < nc && i < s) {
      const T* pq = part + w * (WG / WAVE) * WAVE;
      T sum = pq[lane];
      for (int u = 1; u < WG / WAVE; ++u) sum += pq[u * WAVE + lane];
      cw[(int64_t)(q0 + w) * ldc + a.v_off2 + i] = sum;
    }
  } else {
    for (int j = b0 + w; j < min(b0 + 64, s); j += WG / WAVE) {
      T acc[RCM];
#pragma unroll
      for (int q = 0; q < RCM; ++q) acc[q] = 0;
      for (int i = lane; i < s; i += WAVE) {
        const T x = X[i + (int64_t)j * s];
#pragma unroll
        for (int q = 0; q < RCM; ++q)
          if (q < nc) acc[q] += x * ys[i + q * sp];
      }
#pragma unroll
      for (int q = 0; q < RCM; ++q)
        if (q < nc) {
          const T t = wave_sum(acc[q]);
          if (lane == 0) cw[(int64_t)(q0 + q) * ldc + a.v_off2 + j] = t;
        }
    }
  }
}

template <typename T>
__global__ __launch_bounds__(WG) void k_comp_scatter(const CompApply* __restrict__ A,
                                                     const int32_t* __restrict__ slots, T* __restrict__ y,
                                                     int64_t ldy, const T* __restrict__ cw, int64_t ldc) {
  const CompApply a = A[blockIdx.x];
  const int32_t* sl = slots + a.slot_off;
  for (int i = threadIdx.x; i < a.s; i += WG)
    y[(int64_t)blockIdx.y * ldy + sl[i]] = cw[(int64_t)blockIdx.y * ldc + a.v_off2 + i];
}

// Top node (factor in TF, sweep vectors in TV): mode 0: y <- L^{-T} L^{-1} y;
// mode 1: y <- L L^T y.  With `staged`, the lower triangle of the factor is
// first copied to LDS (ld m + 1), so the sequential steps of the solves read
// LDS instead of waiting on device memory.
template <typename TV, typename T>
__global__ __launch_bounds__(WG) void k_top(const ElimDesc* __restrict__ D, const T* __restrict__ fac,
                                            const int32_t* __restrict__ slots, TV* __restrict__ y, int64_t ldy,
                                            int mode, int staged) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* ys = reinterpret_cast<T*>(smem_raw);
  const ElimDesc d = D[0];
  const int m = d.m;
  T* tmp = ys + m;
  const T* L = fac + d.front_off;
  TV* yv = y + blockIdx.y * ldy;
  const int32_t* sl = slots + d.slot_off;
  for (int i = threadIdx.x; i < m; i += WG) ys[i] = (T)yv[sl[i]];
  if (mode == 0 && staged) {
    T* Ls = tmp + m;
    for (int idx = threadIdx.x; idx < m * m; idx += WG) {
      const int i = idx % m, j = idx / m;
      if (i >= j) Ls[i + j * (m + 1)] = L[idx];
    }
    __syncthreads();
    wg_trsv_lower(Ls, m + 1, m, ys);
    wg_trsv_lower_t(Ls, m + 1, m, ys);
  } else if (mode == 0) {
    __syncthreads();
    wg_trsv_lower(L, m, m, ys);
    wg_trsv_lower_t(L, m, m, ys);
  } else {
    __syncthreads();
    const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
    for (int j = w; j < m; j += WG / WAVE) {
      T acc = 0;
      for (int i = j + lane; i < m; i += WAVE) acc += L[i + (int64_t)j * m] * ys[i];
      acc = wave_sum(acc);
      if (lane == 0) tmp[j] = acc;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < m; i += WG) {
      T acc = 0;
      for (int j = 0; j <= i; ++j) acc += L[i + (int64_t)j * m] * tmp[j];
      ys[i] = acc;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < m; i += WG) yv[sl[i]] = (TV)ys[i];
}

// Permutation between the caller's unknown order and the slot order.
template <typename TI, typename TO>
__global__ void k_gather_perm(const int64_t* __restrict__ perm, int64_t n, const TI* __restrict__ in, int64_t ldi,
                              TO* __restrict__ out, int64_t ldo) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n) out[s + blockIdx.y * ldo] = (TO)in[perm[s] + blockIdx.y * ldi];
}
template <typename TI, typename TO>
__global__ void k_scatter_perm(const int64_t* __restrict__ perm, int64_t n, const TI* __restrict__ in, int64_t ldi,
                               TO* __restrict__ out, int64_t ldo) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n) out[perm[s] + blockIdx.y * ldo] = (TO)in[s + blockIdx.y * ldi];
}

// ---------------------------------------------------------------------------
// CG kernels (FP64)
// ---------------------------------------------------------------------------

// y = A x for nrhs columns, G lanes per row (the row's entries strided over
// the group, summed with shuffles), the matrix read once for up to 8
// columns.  partial[c * gridDim.x + b] = sum over the block's rows of
// x_ic y_ic (fixed order), or nothing when partial is NULL.
template <int G>
__global__ __launch_bounds__(WG) void k_spmv_multi(const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                   const double* __restrict__ va, int64_t n,
                                                   const double* __restrict__ x, int64_t ldx, double* __restrict__ y,
                                                   int64_t ldy, int nrhs, double* __restrict__ partial) {
  constexpr int RC = 8;
  __shared__ double red[WG / WAVE][RC];
  const int tid = threadIdx.x, lane = tid % WAVE, wv = tid / WAVE, g = tid % G;
  const int64_t row = (int64_t)blockIdx.x * (WG / G) + tid / G;
  int64_t e0 = 0, e1 = 0;
  if (row < n) {
    e0 = rp[row];
    e1 = rp[row + 1];
  }
  for (int c0 = 0; c0 < nrhs; c0 += RC) {
    const int nc = min(RC, nrhs - c0);
    const double* xc = x + (int64_t)c0 * ldx;
    double acc[RC];
#pragma unroll
    for (int j = 0; j < RC; ++j) acc[j] = 0;
    // UE entries of the lane at a time, their loads issued first (clamped
    // indices; the entries past the row's end add nothing), accumulated in
    // the lane's entry order
    constexpr int UE = 4;
    for (int64_t eb = e0 + g; eb < e1; eb += (int64_t)G * UE) {
      double a[UE];
      int64_t col[UE];
#pragma unroll
      for (int u = 0; u < UE; ++u) {
        const int64_t e = min(eb + (int64_t)u * G, e1 - 1);
        a[u] = va[e];
        col[u] = ci[e];
      }
#pragma unroll
      for (int u = 0; u < UE; ++u) {
        const bool ok = eb + (int64_t)u * G < e1;
#pragma unroll
        for (int j = 0; j < RC; ++j)
          if (j < nc) {
            const double xv = xc[col[u] + j * ldx];
            if (ok) acc[j] += a[u] * xv;
          }
      }
    }
#pragma unroll
    for (int j = 0; j < RC; ++j)
#pragma unroll
      for (int o = G / 2; o > 0; o >>= 1) acc[j] += __shfl_xor(acc[j], o, WAVE);
    double d[RC];
#pragma unroll
    for (int j = 0; j < RC; ++j) {
      d[j] = 0;
      if (j < nc && row < n && g == 0) {
        y[row + (int64_t)(c0 + j) * ldy] = acc[j];
        d[j] = acc[j] * xc[row + j * ldx];
      }
    }
    if (partial) {
#pragma unroll
      for (int j = 0; j < RC; ++j)
        if (j < nc) {
          const double sj = wave_sum(d[j]);
          if (lane == 0) red[wv][j] = sj;
        }
      __syncthreads();
      if (tid < nc) {
        double sum = 0;
        for (int w = 0; w < WG / WAVE; ++w) sum += red[w][tid];
        partial[(int64_t)(c0 + tid) * gridDim.x + blockIdx.x] = sum;
      }
      __syncthreads();
    }
  }
}

// partial[b] = sum over the block of a_i * b_i.
__global__ __launch_bounds__(WG) void k_dot_partial(const double* __restrict__ a, int64_t lda,
                                                    const double* __restrict__ b, int64_t ldb, int64_t n,
                                                    double* __restrict__ partial) {
  __shared__ double red[WG / WAVE];
  const double* av = a + blockIdx.y * lda;
  const double* bv = b + blockIdx.y * ldb;
  double acc = 0;
  for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * WG) acc += av[i] * bv[i];
  double s = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.y * gridDim.x + blockIdx.x] = s;
}

// out[col * stride] = sum of npart partials (fixed order), one workgroup per column.
__global__ __launch_bounds__(WG) void k_reduce(const double* __restrict__ partial, int npart,
                                               double* __restrict__ out, int stride) {
  __shared__ double red[WG / WAVE];
  const double* p = partial + (int64_t)blockIdx.x * npart;
  double acc = 0;
  for (int i = threadIdx.x; i < npart; i += WG) acc += p[i];
  double s = block_sum(acc, red);
  if (threadIdx.x == 0) out[(int64_t)blockIdx.x * stride] = s;
}

// CG scalars per column.  st layout per column: [rz, pAp, rr, alpha, -, active].
// Every iteration starts from z = M r: with rz = +inf and p = 0 before the
// first one, its beta is 0 and p = z.  beta = rz_new / rz and alpha =
// rz_new / pAp are formed by every workgroup of the vector updates from the
// stored scalars; the x, r update's first workgroup then records rz = rz_new.

// x += alpha p, r -= alpha Ap
__global__ void k_cg_update_xr(double* __restrict__ x, int64_t ldx, double* __restrict__ r, int64_t ldr,
                               const double* __restrict__ p, const double* __restrict__ Ap, int64_t ldp, int64_t n,
                               double* __restrict__ st, const double* __restrict__ rz_new) {
  double* sc = st + 8 * blockIdx.y;
  const bool act = sc[5] != 0.0;
  const double alpha = (act && sc[1] != 0.0) ? rz_new[blockIdx.y] / sc[1] : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc[3] = alpha;
    if (act) sc[0] = rz_new[blockIdx.y];
  }
  if (alpha == 0.0) return;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    x[i + blockIdx.y * ldx] += alpha * p[i + blockIdx.y * ldp];
    r[i + blockIdx.y * ldr] -= alpha * Ap[i + blockIdx.y * ldp];
  }
}
// p = z + beta p
__global__ void k_cg_update_p(double* __restrict__ p, const double* __restrict__ z, int64_t ld, int64_t n,
                              const double* __restrict__ st, const double* __restrict__ rz_new) {
  const double* sc = st + 8 * blockIdx.y;
  if (sc[5] == 0.0) return;
  const double beta = sc[0] != 0.0 ? rz_new[blockIdx.y] / sc[0] : 0.0;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i + blockIdx.y * ld] = z[i + blockIdx.y * ld] + beta * p[i + blockIdx.y * ld];
}

}  // namespace sgf
