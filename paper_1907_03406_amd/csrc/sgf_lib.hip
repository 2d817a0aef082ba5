// C ABI of the SGF library: handles, device memory, the level loop of the
// factorization (Algorithm 4.1), the preconditioner apply (Sec. 4.7), the
// product form (Sec. 2.1) and preconditioned CG (Sec. 7).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <exception>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <functional>
#include <limits>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "sgf.h"
#include "sgf_kernels.hpp"
#include "sgf_plan.hpp"
#include "sgf_tiled.hpp"

namespace {

thread_local std::string g_last_error;

struct SgfError : std::runtime_error {
  sgf_status code;
  SgfError(sgf_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIP_CHECK(expr)                                                                      \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      throw SgfError(SGF_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));       \
  } while (0)

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) {
    o.p = nullptr;
    o.bytes = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      bytes = o.bytes;
      o.p = nullptr;
      o.bytes = 0;
    }
    return *this;
  }
  void ensure(size_t b) {
    if (b <= bytes && p) return;
    release();
    size_t want = b ? b : 16;
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
      p = nullptr;
      bytes = 0;
      (void)hipGetLastError();
      throw SgfError(SGF_ENOMEM, "hipMalloc of " + std::to_string(want) + " bytes failed");
    }
    bytes = want;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <typename T>
  T* as() const {
    return reinterpret_cast<T*>(p);
  }
  ~DevBuf() { release(); }
};

template <typename V>
void upload_direct(DevBuf& b, const std::vector<V>& v, hipStream_t st) {
  b.ensure(v.size() * sizeof(V));
  if (!v.empty()) HIP_CHECK(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(V), hipMemcpyHostToDevice, st));
}

// Pinned staging of the descriptor uploads.  From pageable memory the
// runtime copies synchronously through its own bounce buffer, one table at a
// time; a table placed in pinned memory is queued and the host goes on with
// the next one.  The space is reused once the stream that reads it has been
// synchronized (the factorization synchronizes once per level to read the
// ranks), or after an explicit drain when it is full.
struct Staging {
  unsigned char* p = nullptr;
  size_t cap = 0, used = 0;
  hipStream_t st = nullptr;   // stream of the copies queued since the last reuse point
  bool pending = false;
  static constexpr size_t MAX_TABLE = size_t(64) << 20;   // larger tables go direct
  Staging() = default;
  Staging(const Staging&) = delete;
  Staging& operator=(const Staging&) = delete;
  // wait for the queued copies: on their stream when the caller uses that
  // stream, else on the whole device (the caller's earlier stream may be
  // gone by now)
  void drain(hipStream_t current) {
    if (pending) HIP_CHECK(current == st ? hipStreamSynchronize(st) : hipDeviceSynchronize());
    pending = false;
    used = 0;
  }
  // the caller has synchronized stream s
  void synced(hipStream_t s) {
    if (!pending || s == st) {
      pending = false;
      used = 0;
    }
  }
  // space for `bytes` (256-byte aligned), after the queued copies on stream s
  unsigned char* take(size_t bytes, hipStream_t s) {
    if (pending && s != st) drain(s);
    size_t off = (used + 255) & ~size_t(255);
    if (off + bytes > cap) {
      drain(s);
      off = 0;
      if (bytes > cap) {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
        const size_t want = std::max(bytes, size_t(8) << 20);
        if (hipHostMalloc((void**)&p, want, hipHostMallocDefault) != hipSuccess) {
          p = nullptr;
          (void)hipGetLastError();
          return nullptr;
        }
        cap = want;
      }
    }
    used = off + bytes;
    st = s;
    pending = true;
    return p + off;
  }
  ~Staging() {
    if (pending) (void)hipDeviceSynchronize();
    if (p) (void)hipHostFree(p);
  }
};

// One table to an ensured device buffer, through the staging space unless
// `direct` (or too large for it).
inline void upload_bytes(Staging& S, bool direct, void* dst, const void* src, size_t bytes, hipStream_t st) {
  if (!bytes) return;
  unsigned char* q = direct || bytes > Staging::MAX_TABLE ? nullptr : S.take(bytes, st);
  if (!q) {
    HIP_CHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
    return;
  }
  std::memcpy(q, src, bytes);
  HIP_CHECK(hipMemcpyAsync(dst, q, bytes, hipMemcpyHostToDevice, st));
}

template <typename V>
void upload_staged(Staging& S, bool direct, DevBuf& b, const std::vector<V>& v, hipStream_t st) {
  const size_t bytes = v.size() * sizeof(V);
  b.ensure(bytes);
  upload_bytes(S, direct, b.p, v.data(), bytes, st);
}

// Tables queued while a batch is open (their host vectors unchanged until
// the flush), sent as one blob: one copy and one scatter kernel in place of
// a copy per table.  The device destination is taken when the table is
// queued (the DevBuf object itself may move before the flush, its memory
// does not); a buffer is queued at most once per batch.
struct UploadBatch {
  struct Item {
    void* dst;
    const void* src;
    size_t bytes;
  };
  std::vector<Item> items;
  bool flushed = false;
  void add(DevBuf& b, const void* src, size_t bytes) {
    b.ensure(bytes);
    if (!bytes) return;
    for (auto& it : items)
      if (it.dst == b.p) throw SgfError(SGF_EINVAL, "a device table queued twice in one upload batch");
    items.push_back({b.p, src, bytes});
  }
};

// Algorithmic work of the launches of one level (from the plan).
struct LevelWork {
  double elim_flops = 0, schur_bytes = 0, comp_flops = 0, pair_flops = 0;
  double fwd_bytes = 0, bwd_bytes = 0, fwd_vec = 0, bwd_vec = 0;   // factor part / per-rhs vector part
  double acc_vec = 0, capply_bytes = 0, capply_vec = 0, top_bytes = 0, top_vec = 0;
};

struct LevelDev {
  DevBuf arena, scratch, cf, nbuf, ltphi, tau, phi, rank;
  DevBuf elim, pairs, schur, comp, compnbr, sepacc, sepsrc, capply, slots, nslots;
  DevBuf blkmap, phimap, slotptr, phioff, tb, active, tofcomp, capacc;
  std::vector<sgf::CopyDesc> h_blkmap, h_phimap;
  LevelWork work;
  bool uploaded = false;   // descriptor tables on the device match the plan
  // tiled elimination (large fronts): descriptors, Zt = L_II^{-T}, apply work vector
  bool tiled = false, comp_tiled = false;
  DevBuf elim_order, comp_order;   // work lists of the persistent launches, costliest first
  std::vector<int32_t> h_elim_order, h_comp_order;
  bool elim_uneven = false, comp_uneven = false;
  int64_t c_elems = 0;   // sum of compressed separator sizes (apply vector of the large-separator path)
  DevBuf cw;             // that vector, per right-hand side
  DevBuf tf, zt, uw, ctf;
  std::vector<sgf::TFront> h_tf, h_ctf;
  int64_t z_elems = 0, u_elems = 0;
  int tmax_m = 0, tmax_k = 0, tmax_rm = 0;
  int band_bw = -1, band_m = 0, band_k = 0;   // widest band, largest m and k of the interiors (-1: none)
  int banded_w = 0;                            // 1: the last factorization used the banded elimination
  // level 1 only: every front entry outside the lower band, M_SI, the upper
  // band and the lower separator triangle is known to be zero (after a full
  // clear, kept by the CSR fill and the banded elimination), so the next
  // banded factorization clears just the band and M_SI
  bool front_clean = false;
  bool comp_small = false;                     // compressions by k_compress_small (T_B formed there, in its slot)
  bool capply_small = false;                   // the uploaded apply list uses those slots
  // fronts of the banded elimination grouped by ring width 8 / 16 / 24 / 32
  // (band_ptr[c] .. band_ptr[c + 1] in band_list); band_ok: every front fits one
  std::vector<int32_t> h_band_list;
  int band_ptr[5] = {0, 0, 0, 0, 0};
  bool band_ok = false;
  DevBuf band_list;
  // level-1 inputs of the banded fronts (k_fill_band): the matrix entries
  // that land in the front at band_list position p are fill_ptr[p] ..
  // fill_ptr[p + 1], each with its offset in the front and its CSR index
  // (CSR order); the other entries (pair blocks) for k_fill_rest
  bool fill_ok = false;
  std::vector<int64_t> h_fill_ptr, h_fill_src, h_rest_dst, h_rest_src;
  std::vector<int32_t> h_fill_off;
  DevBuf fill_ptr, fill_off, fill_src, rest_dst, rest_src;
  int64_t fill_rest_n = 0;
  // the one-right-hand-side band solves: fronts of bandwidth <= 16 (the
  // first b1_split), then the others
  std::vector<int32_t> h_b1_list;
  int b1_split = 0;
  DevBuf b1_list;
  DevBuf fixrank;            // low-rank equivalent: the recorded rank of every compression
  // device coarsening into the next level: structure tables (CoarsenPair per
  // pair block, CoarsenSep per separator; coarsen_static once uploaded for
  // the current structure), and each separator's father and first row there
  DevBuf cpairs, cseps, cfather, cloc;
  std::vector<sgf::CoarsenPair> h_cpairs;   // host copies: an upload batch reads them when it is flushed
  std::vector<sgf::CoarsenSep> h_cseps;
  bool coarsen_static = false;
  DevBuf nbroff;             // offset of each neighbour inside an interior's front (nbr_off)
  DevBuf pk;                 // packed factor copies of the banded fronts (ElimDesc::pk_off)
  int64_t pk_elems = 0;
};

struct Profiler {
  bool on = false;
  std::string only;   // non-empty: only launches of this kernel class are timed
  std::vector<sgf_kernel_stat> stats;
  struct Pending {
    int idx;
    hipEvent_t a, b;
    double flops, bytes;
  };
  std::vector<Pending> pending;
  std::vector<Pending> tagged;   // share events with `pending`
  std::vector<hipEvent_t> pool;
  int index(const char* name) {
    for (size_t i = 0; i < stats.size(); ++i)
      if (std::strncmp(stats[i].name, name, sizeof(stats[i].name)) == 0) return (int)i;
    sgf_kernel_stat k{};
    std::snprintf(k.name, sizeof(k.name), "%s", name);
    stats.push_back(k);
    return (int)stats.size() - 1;
  }
  hipEvent_t event() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) throw std::runtime_error("hipEventCreate failed");
    return e;
  }
  // Adds work to a kernel (and its "<name>@L<level>" tag) that is known only
  // after the launch, e.g. once the ranks of a compression are read back.
  void charge(const char* name, int level, double flops, double bytes) {
    if (!on || (!only.empty() && only != name)) return;
    char tag[32];
    std::snprintf(tag, sizeof(tag), "%s@L%d", name, level);
    for (int i : {index(name), index(tag)}) {
      stats[i].flops += flops;
      stats[i].bytes += bytes;
    }
  }
  void drain() {
    for (auto& p : tagged) {
      float ms = 0;
      if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
        auto& k = stats[p.idx];
        k.launches += 1;
        k.ms += ms;
        k.flops += p.flops;
        k.bytes += p.bytes;
      }
    }
    tagged.clear();
    for (auto& p : pending) {
      float ms = 0;
      if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
        auto& k = stats[p.idx];
        k.launches += 1;
        k.ms += ms;
        k.flops += p.flops;
        k.bytes += p.bytes;
      }
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    pending.clear();
  }
  ~Profiler() {
    for (auto& p : pending) {
      (void)hipEventDestroy(p.a);
      (void)hipEventDestroy(p.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

constexpr size_t LDS_BYTES = 64 * 1024;
constexpr size_t LDS_MAX_BYTES = 160 * 1024;   // LDS of one CU on gfx950

// Opt-in host timeline of the factorization (environment SGF_TRACE=1).
struct HostTrace {
  bool on = false;
  std::chrono::steady_clock::time_point t0;
  HostTrace() {
    const char* e = std::getenv("SGF_TRACE");
    on = e && e[0] == '1';
  }
  void start() { t0 = std::chrono::steady_clock::now(); }
  void mark(const char* what, int level) {
    if (!on) return;
    double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    std::fprintf(stderr, "[sgf] %8.3f ms  level %d  %s\n", ms, level, what);
  }
};

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

// One host thread beside the caller's, for host planning that can run while
// the caller's thread queues device work: started on first use, one job at a
// time; wait() returns once the job has ended and rethrows what it threw.
struct HostWorker {
  std::thread th;
  std::mutex m;
  std::condition_variable cv;
  std::function<void()> job;
  bool has_job = false, done = true, quit = false;
  std::exception_ptr err;
  void start(std::function<void()> f) {
    if (!th.joinable()) th = std::thread([this] { loop(); });
    std::lock_guard<std::mutex> g(m);
    job = std::move(f);
    has_job = true;
    done = false;
    err = nullptr;
    cv.notify_all();
  }
  void wait() {
    std::unique_lock<std::mutex> g(m);
    cv.wait(g, [this] { return done; });
    if (err) {
      std::exception_ptr e = err;
      err = nullptr;
      std::rethrow_exception(e);
    }
  }
  void loop() {
    std::unique_lock<std::mutex> g(m);
    for (;;) {
      cv.wait(g, [this] { return has_job || quit; });
      if (quit) return;
      std::function<void()> f = std::move(job);
      has_job = false;
      g.unlock();
      std::exception_ptr e;
      try {
        f();
      } catch (...) {
        e = std::current_exception();
      }
      g.lock();
      err = e;
      done = true;
      cv.notify_all();
    }
  }
  ~HostWorker() {
    {
      std::lock_guard<std::mutex> g(m);
      quit = true;
      cv.notify_all();
    }
    if (th.joinable()) th.join();
  }
};

// Waits for the worker's job on the way out of a scope that started it,
// unless the scope waited itself (active cleared); the job's error is
// dropped there, since another error is already on its way out.
struct WorkerJoin {
  HostWorker* w;
  bool active;
  ~WorkerJoin() {
    if (!active) return;
    try {
      w->wait();
    } catch (...) {
    }
  }
};

struct sgf_handle_s {
  sgf::Plan plan;
  std::vector<int64_t> h_rowptr;
  std::vector<int32_t> h_colidx;
  std::vector<double> h_coords;
  // user near-kernel basis (n x pi, column major, FP64) replacing the
  // monomials of the coordinates; empty: monomials of degree q
  std::vector<double> h_basis;
  // low-rank equivalent (Eq. 7.5): compressions cut at the ranks of the last
  // polynomial factorization, per level and compression
  bool low_rank = false;
  std::vector<std::vector<int32_t>> lr_rank;
  int64_t nnz = 0;
  size_t esz = 8;
  bool dev_static = false;   // CSR structure, perm, coords, fill map on the device
  bool factored = false;
  DevBuf d_perm, d_rowptr, d_colidx, d_vals, d_csrdst, d_coords, d_basis, d_fail;
  DevBuf d_ctr, d_zero_idx;   // work counter of the persistent launches; the one-item list {0}
  std::vector<LevelDev> lev;
  DevBuf y, tscr;
  DevBuf cg_r, cg_z, cg_p, cg_ap, cg_x, cg_part, cg_st, cg_scal;
  int64_t max_t = 0;
  int32_t max_m_all = 0, max_k_all = 0, max_s_all = 0;
  int32_t failed_cluster = -1, failed_level = -1;
  int32_t tiled_rows = 1024;   // levels whose largest front has this many rows go tiled
  // elimination path per level: -1 built-in choice, 0 tiled, 4/8/16/32 one
  // workgroup per front with that panel width (when its LDS panel fits);
  // force_mode overrides all levels (used while tuning)
  std::vector<int32_t> level_mode;
  int32_t force_mode = -1;
  // top node, always factored in FP64: front copy / Cholesky factor, and for
  // the tiled form Zt = L^{-T} and the apply work vector
  DevBuf top64, topz, topu, d_topdesc, d_toptf;
  std::vector<sgf::ElimDesc> h_topdesc;
  std::vector<sgf::TFront> h_toptf;
  bool top_tiled = false;
  int32_t top_R = 0;
  double factor_flops = 0, apply_bytes = 0;
  int64_t factor_entries = 0, factor_bytes = 0, compressed = 0;
  Profiler prof;
  HostTrace trace;
  // apply sweep captured as a HIP graph (one cached instance, keyed by its
  // arguments and the factorization it belongs to), replayed on the caller's
  // stream; captured on a private stream of default priority
  bool use_graph = true;
  bool capturing = false;   // a graph is being recorded: launch directly
  bool band_apply = true;
  bool band1 = true;         // one wavefront per banded front for one right-hand side
  bool apply1 = true;        // one right-hand side on levels of fronts with at most 64 rows: k_apply1
  bool band_elim = true;
  bool small_comp = true;
  bool small_comp_one = false;   // one wavefront per small compression on every level
  int32_t persist_cap = 0;   // > 0: per-level work lists persistent on at most this many workgroups
  int32_t pair_mode = -1;    // coarse couplings: -1 automatic, 0 one workgroup per pair, 1 one wavefront per pair
  // coarsening destinations computed on the device (else host copy maps);
  // switched off: see sgf_set_device_coarsen
  bool device_coarsen = false;
  uint64_t epoch = 0;
  hipStream_t cap_stream = nullptr;
  struct ApplyGraph {
    hipGraphExec_t exec = nullptr;
    int nrhs = 0;
    const double* r = nullptr;
    double* z = nullptr;
    int64_t ldr = 0, ldz = 0;
    bool product = false;
    uint64_t epoch = 0;
  } ag;
  // one PCG iteration (apply, CG scalars and vector updates, SpMV, dots)
  // captured for the buffers and solution pointer it was recorded with
  // (the handle's own CG buffers only, so one graph serves every caller),
  // a few kept for different right-hand-side counts
  struct IterGraph {
    hipGraphExec_t exec = nullptr;
    int nrhs = 0;
    const void* bufs[8] = {};
    uint64_t epoch = 0;
    uint64_t used = 0;
  };
  std::vector<IterGraph> ig;
  uint64_t ig_clock = 0;
  void drop_graph() {
    if (ag.exec) (void)hipGraphExecDestroy(ag.exec);
    ag.exec = nullptr;
    for (auto& g : ig)
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
    ig.clear();
  }
  // second stream (default priority) for independent launches of one level,
  // forked from and joined to the caller's stream with events
  hipStream_t side_stream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  Staging staging;
  UploadBatch* batch = nullptr;   // open upload batch, if any
  DevBuf blob;                    // device copy of the last batch's blob
  hipStream_t blob_st = nullptr;  // stream of the last scatter kernel
  // re-plans the next level while the level loop queues the compressed-
  // separator work (joined before anything reads the next level)
  HostWorker worker;
  ~sgf_handle_s() {
    drop_graph();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (side_stream) (void)hipStreamDestroy(side_stream);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
  }
};

namespace {

// Descriptor tables: staged through pinned memory, direct while a graph is
// being recorded (a recorded copy would read the staging space at replay).
template <typename V>
void upload(sgf_handle h, DevBuf& b, const std::vector<V>& v, hipStream_t st) {
  if (h->batch && !h->capturing) h->batch->add(b, v.data(), v.size() * sizeof(V));
  else upload_staged(h->staging, h->capturing, b, v, st);
}

void flush_batch(sgf_handle h, UploadBatch& B, hipStream_t st) {
  const size_t n = B.items.size();
  auto one_by_one = [&] {
    for (auto& it : B.items) upload_bytes(h->staging, h->capturing, it.dst, it.src, it.bytes, st);
  };
  size_t total = (n * sizeof(sgf::BlobPiece) + 255) & ~size_t(255);
  size_t max_words = 0;
  std::vector<size_t> off(n);
  for (size_t i = 0; i < n; ++i) {
    if (B.items[i].bytes % 4) throw SgfError(SGF_EINVAL, "descriptor table size not a multiple of 4 bytes");
    off[i] = total;
    total += (B.items[i].bytes + 255) & ~size_t(255);
    max_words = std::max(max_words, B.items[i].bytes / 4);
  }
  unsigned char* q = nullptr;
  if (n > 1 && !h->capturing && total <= Staging::MAX_TABLE) {
    // the device blob is rewritten only after the previous scatter read it
    if (h->blob_st && (h->blob_st != st || total > h->blob.bytes))
      HIP_CHECK(h->blob_st == st ? hipStreamSynchronize(st) : hipDeviceSynchronize());
    q = h->staging.take(total, st);
  }
  if (!q) {
    one_by_one();
  } else {
    auto* hp = reinterpret_cast<sgf::BlobPiece*>(q);
    for (size_t i = 0; i < n; ++i) {
      hp[i] = sgf::BlobPiece{off[i], (uint64_t)(uintptr_t)B.items[i].dst, B.items[i].bytes};
      std::memcpy(q + off[i], B.items[i].src, B.items[i].bytes);
    }
    h->blob.ensure(total);
    HIP_CHECK(hipMemcpyAsync(h->blob.p, q, total, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(sgf::k_scatter_blob, dim3((unsigned)n, cdiv((int64_t)max_words, sgf::BLOB_CHUNK)),
                       dim3(sgf::WG), 0, st, h->blob.as<unsigned char>());
    HIP_CHECK(hipGetLastError());
    h->blob_st = st;
  }
  B.flushed = true;
}

// Opens a batch for the uploads of its scope (unless one is open already);
// flush() sends it.  Left without a flush (an error on the way), the levels'
// tables are marked stale so that the next factorization uploads them again.
struct BatchScope {
  sgf_handle h;
  UploadBatch b;
  bool owner;
  explicit BatchScope(sgf_handle hh) : h(hh), owner(hh->batch == nullptr) {
    if (owner) h->batch = &b;
  }
  void flush(hipStream_t st) {
    if (!owner) return;
    h->batch = nullptr;
    flush_batch(h, b, st);
  }
  ~BatchScope() {
    if (!owner) return;
    if (h->batch == &b) h->batch = nullptr;
    if (!b.flushed) {
      for (auto& D : h->lev) D.uploaded = false;
      h->factored = false;
    }
  }
};

sgf_status fail(sgf_status c, const std::string& m) {
  g_last_error = m;
  return c;
}

template <typename F>
sgf_status guard(F&& f) {
  try {
    f();
    return SGF_OK;
  } catch (const SgfError& e) {
    return fail(e.code, e.what());
  } catch (const std::bad_alloc&) {
    return fail(SGF_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(SGF_EINVAL, e.what());
  }
}

// Runs `f` (one kernel launch); when profiling, brackets it with events.
// With level >= 1 the launch is also charged to "<name>@L<level>".
template <typename F>
void launch(sgf_handle h, hipStream_t st, const char* name, double flops, double bytes, F&& f, int level = 0) {
  if (!h->prof.on || (!h->prof.only.empty() && h->prof.only != name)) {
    f();
    return;
  }
  Profiler& p = h->prof;
  int idx = p.index(name);
  hipEvent_t a = p.event(), b = p.event();
  HIP_CHECK(hipEventRecord(a, st));
  f();
  HIP_CHECK(hipEventRecord(b, st));
  p.pending.push_back({idx, a, b, flops, bytes});
  if (level > 0) {
    char tag[32];
    std::snprintf(tag, sizeof(tag), "%s@L%d", name, level);
    p.tagged.push_back({p.index(tag), a, b, flops, bytes});
  }
  if (p.pending.size() > 4096) p.drain();
}

void check_options(const sgf_options* o, int64_t n) {
  if (!o) throw SgfError(SGF_EINVAL, "options pointer is NULL");
  if (o->dim != 2 && o->dim != 3) throw SgfError(SGF_EINVAL, "dim must be 2 or 3");
  int64_t nodes = 1;
  for (int a = 0; a < o->dim; ++a) {
    if (o->grid[a] < 1) throw SgfError(SGF_EINVAL, "grid sizes must be positive");
    nodes *= o->grid[a];
  }
  if (o->dofs_per_node < 1) throw SgfError(SGF_EINVAL, "dofs_per_node must be >= 1");
  if (nodes * o->dofs_per_node != n) throw SgfError(SGF_EINVAL, "n != prod(grid) * dofs_per_node");
  if (o->q < 0 || o->q > 2) throw SgfError(SGF_EINVAL, "q must be 0, 1 or 2");
  if (o->leaf < 2) throw SgfError(SGF_EINVAL, "leaf must be > 1");
  if (o->scheme < SGF_NEST_ALL_ALL || o->scheme > SGF_GEN_ALL_ALL) throw SgfError(SGF_EINVAL, "unknown scheme");
  if (o->precision != SGF_FP64 && o->precision != SGF_FP32 && o->precision != SGF_FP32_BF16N)
    throw SgfError(SGF_EINVAL, "unknown precision");
  if (o->stop_rule != SGF_STOP_ROOT && o->stop_rule != SGF_STOP_PAPER) throw SgfError(SGF_EINVAL, "unknown stop rule");
  if (n >= (int64_t)1 << 31) throw SgfError(SGF_EINVAL, "n must be below 2^31");
}

// Panel width for fronts of up to `rows` rows whose first up to `cols`
// columns are eliminated: the smallest of 4, 8, 16, 32 that covers `cols`
// (narrow panels keep the register-resident diagonal block small), reduced
// until the LDS panel fits beside `extra` elements.
int nb_for(int rows, int cols, size_t esz, int64_t extra = 0) {
  int want = 4;
  while (want < 32 && want < cols) want *= 2;
  for (int nb : {32, 16, 8, 4})
    if (nb <= want && (size_t)std::max<int64_t>(sgf::potrf_lds_elems(rows, nb), extra) * esz <= LDS_BYTES) return nb;
  throw SgfError(SGF_EINVAL, "front of " + std::to_string(rows) + " rows does not fit the LDS panel");
}

template <typename T, bool PERS>
void launch_elim_p(int nb, unsigned grid, size_t lds, hipStream_t st, const sgf::ElimDesc* d, T* arena, int* fail,
                   const int32_t* order, int n, int* ctr) {
  switch (nb) {
    case 32: hipLaunchKernelGGL((sgf::k_elim<T, 32, PERS>), dim3(grid), dim3(sgf::WG), lds, st, d, arena, fail, order, n, ctr); break;
    case 16: hipLaunchKernelGGL((sgf::k_elim<T, 16, PERS>), dim3(grid), dim3(sgf::WG), lds, st, d, arena, fail, order, n, ctr); break;
    case 8: hipLaunchKernelGGL((sgf::k_elim<T, 8, PERS>), dim3(grid), dim3(sgf::WG), lds, st, d, arena, fail, order, n, ctr); break;
    default: hipLaunchKernelGGL((sgf::k_elim<T, 4, PERS>), dim3(grid), dim3(sgf::WG), lds, st, d, arena, fail, order, n, ctr); break;
  }
}
// ctr == nullptr: one workgroup per item; otherwise persistent on the counter.
template <typename T>
void launch_elim(int nb, unsigned grid, size_t lds, hipStream_t st, const sgf::ElimDesc* d, T* arena, int* fail,
                 const int32_t* order, int n, int* ctr) {
  if (ctr) launch_elim_p<T, true>(nb, grid, lds, st, d, arena, fail, order, n, ctr);
  else launch_elim_p<T, false>(nb, grid, lds, st, d, arena, fail, order, n, ctr);
}

// Launch shape of a level's work list of n items: one workgroup per item in
// cluster order, or, when a cap is set, persistent (grid = min(cap, n)
// workgroups taking items costliest first from a counter).  Returns the
// grid; *persist tells which.  Measured on the 2D level-1 fronts the
// one-item launch is the faster (1.17 vs 1.57 ms), so it is the default.
unsigned work_grid(int n, bool* persist, int cap) {
  *persist = cap > 0;
  return (unsigned)std::max<int64_t>(1, *persist ? std::min<int64_t>(cap, n) : n);
}

template <typename T, bool NLDS, bool PERS, typename... A>
void launch_compress_n(int nb, unsigned grid, size_t lds, hipStream_t st, A... args) {
  switch (nb) {
    case 32: hipLaunchKernelGGL((sgf::k_compress<T, 32, NLDS, PERS>), dim3(grid), dim3(sgf::WG), lds, st, args...); break;
    case 16: hipLaunchKernelGGL((sgf::k_compress<T, 16, NLDS, PERS>), dim3(grid), dim3(sgf::WG), lds, st, args...); break;
    case 8: hipLaunchKernelGGL((sgf::k_compress<T, 8, NLDS, PERS>), dim3(grid), dim3(sgf::WG), lds, st, args...); break;
    default: hipLaunchKernelGGL((sgf::k_compress<T, 4, NLDS, PERS>), dim3(grid), dim3(sgf::WG), lds, st, args...); break;
  }
}
template <typename T, typename... A>
void launch_compress(bool nlds, bool pers, int nb, unsigned grid, size_t lds, hipStream_t st, A... args) {
  if (nlds) {
    if (pers) launch_compress_n<T, true, true>(nb, grid, lds, st, args...);
    else launch_compress_n<T, true, false>(nb, grid, lds, st, args...);
  } else {
    if (pers) launch_compress_n<T, false, true>(nb, grid, lds, st, args...);
    else launch_compress_n<T, false, false>(nb, grid, lds, st, args...);
  }
}

void ensure_static(sgf_handle h, hipStream_t st) {
  if (h->dev_static) return;
  upload_direct(h->d_perm, h->plan.perm, st);
  upload_direct(h->d_rowptr, h->h_rowptr, st);
  upload_direct(h->d_colidx, h->h_colidx, st);
  upload_direct(h->d_csrdst, h->plan.csr_dst, st);
  upload_direct(h->d_coords, h->h_coords, st);
  if (!h->h_basis.empty()) upload_direct(h->d_basis, h->h_basis, st);
  h->d_vals.ensure(h->nnz * sizeof(double));
  h->d_fail.ensure(2 * sizeof(int));   // [0] cluster of a non-positive pivot, [1] coarsening range error
  h->d_ctr.ensure(sizeof(int));
  if (!h->d_zero_idx.p) {
    h->d_zero_idx.ensure(sizeof(int32_t));
    HIP_CHECK(hipMemsetAsync(h->d_zero_idx.p, 0, sizeof(int32_t), st));
  }
  h->dev_static = true;
}

// Algorithmic work of eliminating one front (m eliminated, k separator rows)
// whose M_II has lower bandwidth bw (bw = m: dense): band Cholesky, the k rows
// of L_SI against the band factor, and the Schur block (lower half).  With
// bw = m these are m^3/3 + m^2 k + k^2 m.
double elim_flops(double m, double k, double bw) {
  bw = std::min(bw, m);
  return (m * bw * bw - 2.0 / 3.0 * bw * bw * bw) + k * (2.0 * m * bw - bw * bw) + k * k * m;
}
// Factor entries of such a front: the band of L_I and L_SI.
double elim_entries(double m, double k, double bw) {
  bw = std::min(bw, m);
  return m * (bw + 1) - bw * (bw + 1) / 2 + m * k;
}
// HBM bytes of eliminating it: the band of M_II, M_SI and the lower M_SS read
// once and written once.
double elim_bytes(double m, double k, double bw, double e) {
  return 2.0 * e * (elim_entries(m, k, bw) + k * (k + 1) / 2);
}

// Algorithmic work of compressing one separator (s rows, K neighbour rows,
// c = columns of N, numerical rank r, pi basis vectors): Cholesky of M_BB and
// L_B^{-1} M_BX unless already factored, N (Eq. 4.5), the pivoted QR stopped
// at rank r (Eq. 3.3) and Q^T applied to L^T Phi_B (Eq. 3.4).
double comp_flops(double s, double K, double c, double r, double pi, bool prefactored) {
  double f = prefactored ? 0.0 : s * s * s / 3.0 + s * s * K;
  f += s * s * pi + 2.0 * s * K * pi;
  f += 4.0 * s * c * r - 2.0 * r * r * (s + c) + 4.0 * r * r * r / 3.0;
  if (r < s) f += 4.0 * s * r * pi;
  return f;
}
// Its HBM bytes: the front (lower M_BB and M_XB) read, and written back when
// factored here; Phi of B and its neighbours read; L^T Phi_B written (and
// rewritten by Q^T when r < s); the reflectors (s x r) and tau written.
double comp_bytes(double s, double K, double c, double r, double pi, bool prefactored, double e) {
  const double front = s * (s + 1) / 2 + K * s;
  double b = (prefactored ? 1.0 : 2.0) * front + (s + K) * pi + s * pi + s * r + c;
  if (r < s) b += 2.0 * s * pi;
  return b * e;
}

// Whether the interiors of level L are eliminated by the tiled multi-workgroup
// path: fronts at or above the row threshold, or too large for the LDS panel
// of the one-workgroup-per-front kernel.
int level_mode(sgf_handle h, const sgf::Level& L) {
  if (h->force_mode != -1) return h->force_mode;
  const int li = L.t - 1;
  return li < (int)h->level_mode.size() ? h->level_mode[li] : -1;
}

bool panel_fits(int rows, int nb, size_t esz) {
  return (size_t)sgf::potrf_lds_elems(rows, nb) * esz <= LDS_BYTES;
}

// LDS bytes of the one-workgroup apply kernels for fronts of `rows` rows, one rhs.
size_t apply_lds(int rows, size_t esz) {
  return ((size_t)sgf::DB * sgf::DLD + ((rows + 3) & ~3)) * esz;
}

bool level_tiled(sgf_handle h, const sgf::Level& L) {
  if (L.top || L.elim.empty()) return false;
  if (apply_lds(L.max_front_rows, h->esz) > LDS_BYTES) return true;
  const int mode = level_mode(h, L);
  if (mode == 0) return true;
  if (mode >= 8) return !panel_fits(L.max_front_rows, mode, h->esz);
  if (L.max_front_rows >= h->tiled_rows) return true;
  int max_m = 0;
  for (const auto& e : L.elim) max_m = std::max(max_m, e.m);
  try {
    (void)nb_for(L.max_front_rows, max_m, h->esz);
  } catch (const SgfError&) {
    return true;
  }
  return false;
}

// Panel width of the one-workgroup elimination of level L.
int level_nb(sgf_handle h, const sgf::Level& L, int max_m) {
  const int mode = level_mode(h, L);   // 1 (banded) on a level that is not banded: automatic width
  if (mode >= 8 && panel_fits(L.max_front_rows, mode, h->esz)) return mode;
  return nb_for(L.max_front_rows, max_m, h->esz);
}

// Whether a level runs the banded one-wavefront elimination (1) or not (0):
// every interior with lower bandwidth below 32 and at most 64 separator
// rows, the level not tiled, and the level's mode automatic (-1) or banded
// (1).  The fronts are launched in groups of equal ring width.
int banded_w(sgf_handle h, const sgf::Level& L, const LevelDev& D) {
  if (!h->band_elim || L.top || L.elim.empty() || D.tiled || !D.band_ok) return 0;
  const int mode = level_mode(h, L);
  return mode == -1 || mode == 1 ? 1 : 0;
}

// Descriptors and buffers of a tiled level: Zt (m x m per front) and the
// apply work vector (m per front and right-hand side).
void build_tiled(sgf_handle h, const sgf::Level& L, LevelDev& D, hipStream_t st) {
  D.h_tf.clear();
  D.z_elems = D.u_elems = 0;
  D.tmax_m = D.tmax_k = D.tmax_rm = 0;
  for (const auto& e : L.elim) {
    sgf::TFront f{};
    f.f_off = e.front_off;
    f.z_off = D.z_elems;
    f.u_off = D.u_elems;
    f.slot_off = e.slot_off;
    f.nslot_off = e.nslot_off;
    f.t_off = e.t_off;
    f.R = e.m + e.k;
    f.m = e.m;
    f.cluster = e.cluster;
    f.zrows = e.m;
    D.z_elems += (int64_t)e.m * e.m;
    D.u_elems += e.m;
    D.tmax_m = std::max(D.tmax_m, e.m);
    D.tmax_k = std::max(D.tmax_k, e.k);
    D.tmax_rm = std::max(D.tmax_rm, 2 * e.m + e.k);
    D.h_tf.push_back(f);
  }
  if ((size_t)(((D.tmax_m + 3) & ~3) + sgf::WG) * h->esz > LDS_BYTES || (size_t)D.tmax_k * h->esz > LDS_BYTES)
    throw SgfError(SGF_EINVAL, "front too large for the tiled apply kernels");
  upload(h, D.tf, D.h_tf, st);
  D.zt.ensure(std::max<int64_t>(D.z_elems, 1) * h->esz);
}

// Upload the descriptor tables of level index li and size its buffers.
// Level-1 matrix entries split by destination: those in a banded front go
// to that front's list (k_fill_band writes them after clearing the front's
// band), the rest (pair blocks) to one list for k_fill_rest.  Only when every
// front is banded and fits the 32-bit in-front offsets.
void build_fill_lists(sgf_handle h, const sgf::Level& L, LevelDev& D, hipStream_t st) {
  D.fill_ok = false;
  if (!D.band_ok || D.h_band_list.empty()) return;
  const std::vector<int64_t>& dst = h->plan.csr_dst;
  const int nb = (int)D.h_band_list.size();
  std::vector<std::pair<int64_t, int>> fo(nb);   // (front offset, band position)
  for (int p = 0; p < nb; ++p) {
    const auto& e = L.elim[D.h_band_list[p]];
    const int64_t R = (int64_t)e.m + e.k;
    if (R * R >= ((int64_t)1 << 31)) return;
    fo[p] = {e.front_off, p};
  }
  std::sort(fo.begin(), fo.end());
  // band position of an arena offset inside a banded front, else -1
  auto front_of = [&](int64_t d) {
    auto it = std::upper_bound(fo.begin(), fo.end(), std::make_pair(d, std::numeric_limits<int>::max()));
    if (it == fo.begin()) return -1;
    --it;
    const auto& e = L.elim[D.h_band_list[it->second]];
    const int64_t R = (int64_t)e.m + e.k;
    return d < it->first + R * R ? it->second : -1;
  };
  const int64_t nnz = (int64_t)dst.size();
  std::vector<int32_t> pos(nnz, -1);
  D.h_fill_ptr.assign(nb + 1, 0);
  D.h_rest_dst.clear();
  D.h_rest_src.clear();
  for (int64_t e = 0; e < nnz; ++e) {
    if (dst[e] < 0) continue;
    pos[e] = front_of(dst[e]);
    if (pos[e] >= 0) {
      ++D.h_fill_ptr[pos[e] + 1];
    } else {
      D.h_rest_dst.push_back(dst[e]);
      D.h_rest_src.push_back(e);
    }
  }
  for (int p = 0; p < nb; ++p) D.h_fill_ptr[p + 1] += D.h_fill_ptr[p];
  D.h_fill_off.assign(D.h_fill_ptr[nb], 0);
  D.h_fill_src.assign(D.h_fill_ptr[nb], 0);
  std::vector<int64_t> cur(D.h_fill_ptr.begin(), D.h_fill_ptr.end() - 1);
  for (int64_t e = 0; e < nnz; ++e) {
    if (pos[e] < 0) continue;
    const int64_t q = cur[pos[e]]++;
    D.h_fill_off[q] = (int32_t)(dst[e] - L.elim[D.h_band_list[pos[e]]].front_off);
    D.h_fill_src[q] = e;
  }
  // keep the device lists non-empty (valid pointers for empty launches)
  if (D.h_rest_dst.empty()) {
    D.h_rest_dst.push_back(0);
    D.h_rest_src.push_back(0);
    D.fill_rest_n = 0;
  } else {
    D.fill_rest_n = (int64_t)D.h_rest_dst.size();
  }
  if (D.h_fill_off.empty()) {
    D.h_fill_off.push_back(0);
    D.h_fill_src.push_back(0);
  }
  upload(h, D.fill_ptr, D.h_fill_ptr, st);
  upload(h, D.fill_off, D.h_fill_off, st);
  upload(h, D.fill_src, D.h_fill_src, st);
  upload(h, D.rest_dst, D.h_rest_dst, st);
  upload(h, D.rest_src, D.h_rest_src, st);
  D.fill_ok = true;
}

void upload_level(sgf_handle h, int li, hipStream_t st) {
  sgf::Level& L = h->plan.levels[li];
  if ((int)h->lev.size() <= li) h->lev.resize(li + 1);
  LevelDev& D = h->lev[li];
  if (D.uploaded) return;
  D.uploaded = true;
  D.front_clean = false;
  const size_t e = h->esz;
  D.arena.ensure((L.front_elems + L.blk_elems) * e);
  D.scratch.ensure(L.scratch_elems * e);
  D.cf.ensure(L.cf_elems * e);
  D.nbuf.ensure(L.n_elems * e);
  D.ltphi.ensure(L.ltphi_elems * e);
  D.tau.ensure(L.tau_elems * e);
  D.phi.ensure(L.phi_elems * e);
  D.rank.ensure(std::max<size_t>(L.comp.size(), 1) * sizeof(int));
  D.band_bw = -1;
  D.band_m = D.band_k = 0;
  for (const auto& e : L.elim) {
    D.band_bw = std::max(D.band_bw, std::min(e.bw, std::max(e.m - 1, 0)));
    D.band_m = std::max(D.band_m, e.m);
    D.band_k = std::max(D.band_k, e.k);
  }
  {
    // ring-width classes of the banded elimination
    std::vector<int32_t> cls[4];
    D.band_ok = !L.elim.empty();
    for (size_t f = 0; f < L.elim.size(); ++f) {
      const auto& e = L.elim[f];
      const int b = std::min(e.bw, std::max(e.m - 1, 0));
      const int c = b < 8 ? 0 : b < 16 ? 1 : b < 24 ? 2 : b < 32 ? 3 : -1;
      if (c < 0 || e.k > sgf::BE_KMAX) {
        D.band_ok = false;
        break;
      }
      cls[c].push_back((int32_t)f);
    }
    D.h_band_list.clear();
    D.band_ptr[0] = 0;
    for (int c = 0; c < 4; ++c) {
      if (D.band_ok) D.h_band_list.insert(D.h_band_list.end(), cls[c].begin(), cls[c].end());
      D.band_ptr[c + 1] = (int)D.h_band_list.size();
    }
    if (D.band_ok) upload(h, D.band_list, D.h_band_list, st);
    if (li == 0) build_fill_lists(h, L, D, st);
    D.h_b1_list.clear();
    if (D.band_ok) {
      for (int pass = 0; pass < 2; ++pass) {
        for (size_t f = 0; f < L.elim.size(); ++f) {
          const auto& e = L.elim[f];
          if ((std::min(e.bw, std::max(e.m - 1, 0)) <= 16) == (pass == 0)) D.h_b1_list.push_back((int32_t)f);
        }
        if (pass == 0) D.b1_split = (int)D.h_b1_list.size();
      }
      upload(h, D.b1_list, D.h_b1_list, st);
    }
    // packed copies for the apply sweeps, 64-element aligned
    D.pk_elems = 0;
    for (auto& e : L.elim) {
      if (D.band_ok) {
        e.pk_off = D.pk_elems;
        D.pk_elems += sgf::band_pk_elems(e.m, e.k, std::min(e.bw, std::max(e.m - 1, 0)));
      } else {
        e.pk_off = -1;
      }
    }
  }
  upload(h, D.elim, L.elim, st);
  upload(h, D.pairs, L.pairs, st);
  upload(h, D.schur, L.schur, st);
  upload(h, D.comp, L.comp, st);
  upload(h, D.compnbr, L.comp_nbr, st);
  upload(h, D.sepacc, L.sepacc, st);
  upload(h, D.sepsrc, L.sepacc_src, st);
  upload(h, D.slots, L.slots, st);
  upload(h, D.nslots, L.nslots, st);
  upload(h, D.nbroff, L.nbr_off, st);
  upload(h, D.slotptr, L.slot_ptr, st);
  upload(h, D.phioff, L.phi_off, st);
  D.tiled = level_tiled(h, L);
  if (D.tiled) build_tiled(h, L, D, st);

  {
    // work lists of the persistent launches: costliest first when the costs
    // differ by more than 2x (longest-processing-time order), else cluster
    // order (memory locality); each cost evaluated once
    std::vector<double> cost;
    auto order = [&cost](std::vector<int32_t>& o, bool* uneven) {
      const size_t n = cost.size();
      o.resize(n);
      for (size_t i = 0; i < n; ++i) o[i] = (int32_t)i;
      double lo = 0, hi = 0;
      for (size_t i = 0; i < n; ++i) {
        lo = i ? std::min(lo, cost[i]) : cost[i];
        hi = i ? std::max(hi, cost[i]) : cost[i];
      }
      *uneven = hi > 2 * lo;
      if (*uneven) std::stable_sort(o.begin(), o.end(), [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
    };
    cost.resize(L.elim.size());
    for (size_t a = 0; a < L.elim.size(); ++a) cost[a] = elim_flops(L.elim[a].m, L.elim[a].k, L.elim[a].bw);
    order(D.h_elim_order, &D.elim_uneven);
    upload(h, D.elim_order, D.h_elim_order, st);
    cost.resize(L.comp.size());
    for (size_t c = 0; c < L.comp.size(); ++c)
      cost[c] = (double)L.comp[c].s * L.comp[c].s * (L.comp[c].s + L.comp[c].K + L.comp[c].c);
    order(D.h_comp_order, &D.comp_uneven);
    upload(h, D.comp_order, D.h_comp_order, st);
  }
  // compression fronts [M_BB ; M_XB] too large for the one-workgroup panel:
  // their Cholesky / triangular solve goes through the tiled kernels
  D.comp_tiled = false;
  if (!L.comp.empty()) {
    int max_s = 0, max_rows = 0;
    for (const auto& d : L.comp) {
      max_s = std::max(max_s, d.s);
      max_rows = std::max(max_rows, d.s + d.K);
    }
    D.comp_tiled = max_rows >= h->tiled_rows;
    if (!D.comp_tiled) {
      try {
        (void)nb_for(max_rows, max_s, h->esz);
      } catch (const SgfError&) {
        D.comp_tiled = true;
      }
    }
    if (D.comp_tiled) {
      D.h_ctf.clear();
      for (const auto& d : L.comp) {
        sgf::TFront f{};
        f.f_off = d.cf_off;
        f.R = d.s + d.K;
        f.m = d.s;
        f.cluster = d.cluster;
        f.zrows = 0;
        D.h_ctf.push_back(f);
      }
      upload(h, D.ctf, D.h_ctf, st);
    }
  }
}

template <typename T>
void zero(DevBuf& b, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  unsigned g = std::min<int64_t>(cdiv(n, sgf::WG), 65536);
  hipLaunchKernelGGL(sgf::k_zero<T>, dim3(g), dim3(sgf::WG), 0, st, b.as<T>(), n);
}

// Lanes per CSR row of the SpMV: about half the mean row length, 4..64.
int spmv_group(sgf_handle h) {
  const double avg = (double)h->nnz / std::max<int64_t>(h->plan.n, 1);
  int g = 1;
  while (g < 64 && 4 * g < avg) g *= 2;
  return g;
}

unsigned spmv_blocks(sgf_handle h) { return cdiv(h->plan.n, sgf::WG / spmv_group(h)); }

void spmv_launch(sgf_handle h, const double* x, int64_t ldx, double* y, int64_t ldy, int nrhs, double* partial,
                 hipStream_t st) {
  const int64_t n = h->plan.n;
  const unsigned nb = spmv_blocks(h);
  const int64_t* rp = h->d_rowptr.as<int64_t>();
  const int32_t* ci = h->d_colidx.as<int32_t>();
  const double* va = h->d_vals.as<double>();
  switch (spmv_group(h)) {
    case 1: hipLaunchKernelGGL(sgf::k_spmv_multi<1>, dim3(nb), dim3(sgf::WG), 0, st, rp, ci, va, n, x, ldx, y, ldy, nrhs, partial); break;
    case 2: hipLaunchKernelGGL(sgf::k_spmv_multi<2>, dim3(nb), dim3(sgf::WG), 0, st, rp, ci, va, n, x, ldx, y, ldy, nrhs, partial); break;
    case 4: hipLaunchKernelGGL(sgf::k_spmv_multi<4>, dim3(nb), dim3(sgf::WG), 0, st, rp, ci, va, n, x, ldx, y, ldy, nrhs, partial); break;
    case 8: hipLaunchKernelGGL(sgf::k_spmv_multi<8>, dim3(nb), dim3(sgf::WG), 0, st, rp, ci, va, n, x, ldx, y, ldy, nrhs, partial); break;
    case 16: hipLaunchKernelGGL(sgf::k_spmv_multi<16>, dim3(nb), dim3(sgf::WG), 0, st, rp, ci, va, n, x, ldx, y, ldy, nrhs, partial); break;
    case 32: hipLaunchKernelGGL(sgf::k_spmv_multi<32>, dim3(nb), dim3(sgf::WG), 0, st, rp, ci, va, n, x, ldx, y, ldy, nrhs, partial); break;
    default: hipLaunchKernelGGL(sgf::k_spmv_multi<64>, dim3(nb), dim3(sgf::WG), 0, st, rp, ci, va, n, x, ldx, y, ldy, nrhs, partial); break;
  }
}

int check_fail(sgf_handle h, hipStream_t st) {
  int f[2] = {-1, 0};
  HIP_CHECK(hipMemcpyAsync(f, h->d_fail.p, sizeof(f), hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  h->staging.synced(st);
  if (h->blob_st == st) h->blob_st = nullptr;   // its last scatter has run
  if (f[1] != 0) throw SgfError(SGF_EINVAL, "coarsening: a block destination fell outside its buffer (nothing copied)");
  return f[0];
}

void account_level(sgf_handle h, const sgf::Level& L, LevelWork& W) {
  W = LevelWork{};
  const double e = (double)h->esz;
  for (const auto& d : L.elim) {
    double m = d.m, k = d.k, tri = m * (m + 1) / 2, ent = elim_entries(m, k, d.bw);
    W.elim_flops += elim_flops(m, k, d.bw);
    h->factor_entries += (int64_t)ent;
    if (L.top) {
      W.top_bytes += tri * e;
      W.top_vec += 2 * m * e + 4 * m;
    } else {
      W.fwd_bytes += ent * e;
      W.bwd_bytes += ent * e;
      W.fwd_vec += (2 * m + k) * e + 4 * m;
      W.bwd_vec += (2 * m + k) * e + 4 * (m + k);
    }
  }
  for (const auto& a : L.sepacc) W.acc_vec += (double)a.s * (a.c_cnt + 2) * e + 4.0 * a.s + 8.0 * a.c_cnt;
  const int pi = h->plan.pi;
  for (size_t c = 0; c < L.comp.size(); ++c) {
    const auto& d = L.comp[c];
    double s = d.s, K = d.K, cc = d.c, r = L.rank.empty() ? 0 : L.rank[c];
    W.comp_flops += s * s * s / 3.0 + s * s * K + s * s * pi + 2.0 * s * K * pi;
    W.comp_flops += 4.0 * s * cc * r - 2.0 * r * r * (s + cc) + 4.0 * r * r * r / 3.0;
  }
  for (const auto& a : L.capply) {
    double s = a.s;
    h->factor_entries += (int64_t)(s * s);
    W.capply_bytes += s * s * e;
    W.capply_vec += 2 * s * e + 4 * s;
  }
  for (const auto& p : L.pairs) {
    W.schur_bytes += (double)p.s_a * p.s_b * (p.c_cnt + 2) * e;
    if (p.a == p.b || L.rank.empty()) continue;
    int ra = p.ca >= 0 && L.rank[p.ca] < p.s_a ? L.rank[p.ca] : p.s_a;
    int rb = p.cb >= 0 && L.rank[p.cb] < p.s_b ? L.rank[p.cb] : p.s_b;
    if (ra < p.s_a) W.pair_flops += 4.0 * (double)p.s_a * ra * p.s_b;
    if (rb < p.s_b) W.pair_flops += (double)p.s_b * p.s_b * ra + 4.0 * (double)p.s_b * rb * ra;
  }
  h->factor_flops += W.elim_flops + W.comp_flops + W.pair_flops;
  h->apply_bytes += W.fwd_bytes + W.bwd_bytes + W.fwd_vec + W.bwd_vec + W.acc_vec * 2 + 2 * W.capply_bytes +
                    2 * W.capply_vec + W.top_bytes + W.top_vec;
}

// Tiled elimination of the fronts `tf` (factor buffer fb, Zt buffer zb): one
// panel launch and one update launch per 64 eliminated columns, then the
// Schur contraction.  Flops are attributed per launch from the front sizes.
template <typename T>
void tiled_factor(sgf_handle h, hipStream_t st, const std::vector<sgf::TFront>& tf, const sgf::TFront* dtf, T* fb,
                  T* zb, int level, const char* kind, bool schur = true) {
  const unsigned nf = (unsigned)tf.size();
  if (nf == 0) return;
  int max_m = 0, max_rm = 0;
  double zelems = 0;
  for (const auto& f : tf) {
    max_m = std::max(max_m, f.m);
    max_rm = std::max(max_rm, f.R + f.zrows);
    zelems += (double)f.zrows * f.m;
  }
  const double e = sizeof(T);
  const std::string k(kind);
  const std::string n_init = k + "_zinit", n_panel = k + "_panel", n_upd = k + "_update", n_schur = k + "_schur";
  if (zelems > 0)
    launch(h, st, n_init.c_str(), 0, zelems * e, [&] {
      hipLaunchKernelGGL(sgf::k_tinit<T>, dim3(std::min<unsigned>(cdiv(max_m * (int64_t)max_m, sgf::WG), 1024), nf),
                         dim3(sgf::WG), 0, st, dtf, zb);
    }, level);
  const unsigned g1 = cdiv(max_rm, sgf::TROWS);
  for (int p = 0; p * sgf::TB < max_m; ++p) {
    const int c0 = p * sgf::TB;
    double pfl = 0, ufl = 0;
    unsigned g2 = 0;
    for (const auto& f : tf) {
      if (c0 >= f.m) continue;
      const double w = std::min(sgf::TB, f.m - c0);
      pfl += w * w * w / 3.0 + (double)(f.R - c0 - w) * w * w;
      const int c1 = c0 + sgf::TB;
      if (c1 < f.m) {
        const int nj = (int)cdiv(f.m, sgf::TB) - p - 1, nrt = (int)cdiv(f.R, sgf::TB) + (f.zrows > 0 ? p + 1 : 0);
        g2 = std::max<unsigned>(g2, (unsigned)(nj * nrt));
        const double cols = f.m - c1, rows = f.R - c1;
        ufl += 2.0 * sgf::TB * (rows * cols - cols * cols / 2.0);
      }
    }
    launch(h, st, n_panel.c_str(), 0, 0, [&] {
      hipLaunchKernelGGL(sgf::k_tdiag<T>, dim3(nf), dim3(sgf::WAVE), 0, st, dtf, p, fb, h->d_fail.as<int>());
    }, level);
    launch(h, st, n_panel.c_str(), pfl, 0, [&] {
      hipLaunchKernelGGL(sgf::k_tpanel<T>, dim3(g1, nf), dim3(sgf::WG), 0, st, dtf, p, fb, zb);
    }, level);
    if (g2)
      launch(h, st, n_upd.c_str(), ufl, 0, [&] {
        hipLaunchKernelGGL(sgf::k_tupdate<T>, dim3(g2, nf), dim3(sgf::WG), 0, st, dtf, p, fb, zb);
      }, level);
  }
  unsigned g3 = 0;
  double sfl = 0;
  for (const auto& f : tf) {
    const int k = f.R - f.m, nst = (int)cdiv(k, sgf::TB);
    g3 = std::max<unsigned>(g3, (unsigned)(nst * nst));
    sfl += (double)k * k * f.m;
  }
  if (g3 && schur)
    launch(h, st, n_schur.c_str(), sfl, 0, [&] {
      hipLaunchKernelGGL(sgf::k_tschur<T>, dim3(g3, nf), dim3(sgf::WG), 0, st, dtf, fb);
    }, level);
}

// The top node is always factored in FP64 (from a copy of its front), by
// one workgroup when small, else by the tiled path, which also forms Zt.
template <typename T>
void factor_top(sgf_handle h, const sgf::Level& L, LevelDev& D, hipStream_t st) {
  const sgf::ElimDesc& e0 = L.elim[0];
  const int R = e0.m;
  h->top_R = R;
  h->top_tiled = false;
  if (R == 0) return;
  const int64_t RR = (int64_t)R * R;
  h->top64.ensure(RR * sizeof(double));
  launch(h, st, "top_convert", 0, RR * (8.0 + sizeof(T)), [&] {
    hipLaunchKernelGGL((sgf::k_convert<T, double>), dim3(std::min<unsigned>(cdiv(RR, sgf::WG), 4096)), dim3(sgf::WG),
                       0, st, D.arena.as<T>() + e0.front_off, h->top64.as<double>(), RR);
  }, L.t);
  h->h_topdesc.assign(1, e0);
  h->h_topdesc[0].front_off = 0;
  upload(h, h->d_topdesc, h->h_topdesc, st);
  h->top_tiled = R > 256 || R >= h->tiled_rows;
  if (h->top_tiled) {
    if ((size_t)(((R + 3) & ~3) + sgf::WG) * sizeof(double) > LDS_BYTES)
      throw SgfError(SGF_EINVAL, "top node of " + std::to_string(R) + " rows is too large for the tiled apply");
    sgf::TFront f{};
    f.zrows = R;
    f.slot_off = e0.slot_off;
    f.nslot_off = e0.nslot_off;
    f.t_off = e0.t_off;
    f.R = R;
    f.m = R;
    f.cluster = e0.cluster;
    h->h_toptf.assign(1, f);
    upload(h, h->d_toptf, h->h_toptf, st);
    h->topz.ensure(RR * sizeof(double));
    tiled_factor<double>(h, st, h->h_toptf, h->d_toptf.as<sgf::TFront>(), h->top64.as<double>(),
                         h->topz.as<double>(), L.t, "top");
  } else {
    const int nb = nb_for(R, R, sizeof(double));
    const size_t lds = (size_t)sgf::potrf_lds_elems(R, nb) * sizeof(double);
    launch(h, st, "top_chol", (double)R * R * R / 3.0, 0, [&] {
      launch_elim<double>(nb, 1, lds, st, h->d_topdesc.as<sgf::ElimDesc>(), h->top64.as<double>(),
                          h->d_fail.as<int>(), h->d_zero_idx.as<int32_t>(), 1, nullptr);
    }, L.t);
  }
}

template <typename T>
void factor_numeric(sgf_handle h, const double* vals, hipStream_t st) {
  sgf::Plan& P = h->plan;
  h->trace.start();
  ensure_static(h, st);
  // levels above the first depend on the ranks: a planned level is reused as
  // long as the ranks below it come out the same as when it was planned
  if ((int)P.levels.size() > (int)h->lev.size()) {
    P.levels.resize(1);
    P.parts.resize(1);
  }
  h->factored = false;
  ++h->epoch;
  h->drop_graph();
  h->factor_flops = 0;
  h->apply_bytes = 0;
  h->factor_entries = 0;
  h->compressed = 0;
  h->failed_cluster = h->failed_level = -1;
  h->max_t = 0;
  h->max_m_all = h->max_k_all = h->max_s_all = 0;
  if (vals != h->d_vals.as<double>())
    HIP_CHECK(hipMemcpyAsync(h->d_vals.p, vals, h->nnz * sizeof(double), hipMemcpyDefault, st));
  const int init[2] = {-1, 0};
  HIP_CHECK(hipMemcpyAsync(h->d_fail.p, init, sizeof(init), hipMemcpyHostToDevice, st));
  const double e = (double)sizeof(T);
  // ---- level 1 inputs ---------------------------------------------------------
  {
    BatchScope bs(h);
    upload_level(h, 0, st);
    bs.flush(st);
  }
  {
    sgf::Level& L = P.levels[0];
    LevelDev& D = h->lev[0];
    const int64_t ne = L.front_elems + L.blk_elems;
    const bool band_inputs = D.front_clean && banded_w(h, L, D) > 0;
    const bool fused = band_inputs && D.fill_ok;
    if (band_inputs) {
      double zb = (double)L.blk_elems * e;
      for (const auto& d : L.elim) zb += (double)d.m * (std::min(d.bw, std::max(d.m - 1, 0)) + 1 + d.k) * e;
      launch(h, st, "zero", 0, zb, [&] {
        if (L.blk_elems > 0) {
          const unsigned g = std::min<int64_t>(cdiv(L.blk_elems, sgf::WG), 65536);
          hipLaunchKernelGGL(sgf::k_zero<T>, dim3(g), dim3(sgf::WG), 0, st, D.arena.as<T>() + L.front_elems,
                             L.blk_elems);
        }
        if (!fused)
          hipLaunchKernelGGL(sgf::k_zero_band<T>, dim3((unsigned)D.h_band_list.size()), dim3(sgf::WG), 0, st,
                             D.elim.as<sgf::ElimDesc>(), D.band_list.as<int32_t>(), D.arena.as<T>());
      }, L.t);
    } else {
      launch(h, st, "zero", 0, ne * e, [&] { zero<T>(D.arena, ne, st); }, L.t);
    }
    // set again once the banded elimination of this factorization is queued
    D.front_clean = false;
    if (fused) {
      // the pair-block entries first, while the blocks just cleared are still
      // cached; then, per banded front, the band and M_SI cleared and the
      // front's own entries written in one pass
      if (D.fill_rest_n > 0)
        launch(h, st, "fill_csr", 0, D.fill_rest_n * (24.0 + e), [&] {
          hipLaunchKernelGGL(sgf::k_fill_rest<T>, dim3(cdiv(D.fill_rest_n, 4 * sgf::WG)), dim3(sgf::WG), 0, st,
                             h->d_vals.as<double>(), D.rest_dst.as<int64_t>(), D.rest_src.as<int64_t>(),
                             D.fill_rest_n, D.arena.as<T>());
        });
      launch(h, st, "fill_band", 0, (double)(D.h_fill_ptr.back()) * (20.0 + e), [&] {
        hipLaunchKernelGGL(sgf::k_fill_band<T>, dim3((unsigned)D.h_band_list.size()), dim3(sgf::WG), 0, st,
                           D.elim.as<sgf::ElimDesc>(), D.band_list.as<int32_t>(), D.fill_ptr.as<int64_t>(),
                           D.fill_off.as<int32_t>(), D.fill_src.as<int64_t>(), h->d_vals.as<double>(),
                           D.arena.as<T>());
      }, L.t);
    } else {
      launch(h, st, "fill_csr", 0, h->nnz * (16.0 + e), [&] {
        hipLaunchKernelGGL(sgf::k_fill_csr<T>, dim3(cdiv(h->nnz, sgf::WG)), dim3(sgf::WG), 0, st,
                           h->d_vals.as<double>(), h->d_csrdst.as<int64_t>(), h->nnz, D.arena.as<T>());
      });
    }
    sgf::PhiInit pin{};
    for (int a = 0; a < 3; ++a) {
      pin.lo[a] = P.cmin[a];
      pin.sc[a] = P.cmax[a] > P.cmin[a] ? 2.0 / (P.cmax[a] - P.cmin[a]) : 0.0;
    }
    pin.dim = P.opt.dim;
    pin.q = P.opt.q;
    pin.dpn = P.opt.dpn;
    pin.pi = P.pi;
    pin.p0 = P.pi / P.opt.dpn;
    if (!L.cell.empty() && !h->h_basis.empty())
      launch(h, st, "phi_init", 0, (double)P.n * (P.pi * (e + 8) + 8), [&] {
        hipLaunchKernelGGL(sgf::k_phi_user<T>, dim3((unsigned)L.cell.size()), dim3(sgf::WG), 0, st,
                           D.slotptr.as<int64_t>(), D.phioff.as<int64_t>(), h->d_perm.as<int64_t>(),
                           h->d_basis.as<double>(), P.n, P.pi, D.phi.as<T>());
      });
    else if (!L.cell.empty())
      launch(h, st, "phi_init", 0, (double)P.n * (P.pi * e + 8 + 8 * P.opt.dim), [&] {
        hipLaunchKernelGGL(sgf::k_phi_init<T>, dim3((unsigned)L.cell.size()), dim3(sgf::WG), 0, st,
                           D.slotptr.as<int64_t>(), D.phioff.as<int64_t>(), h->d_perm.as<int64_t>(),
                           h->d_coords.as<double>(), pin, D.phi.as<T>());
      });
  }
  h->trace.mark("level-1 inputs queued", 1);
  // ---- level loop (Algorithm 4.1) --------------------------------------------
  // the work counters of a level are summed on the host while the GPU runs
  // the level after it (off the path between the rank read-back and the
  // next launches)
  int acct = -1;
  auto account_pending = [&] {
    if (acct < 0) return;
    account_level(h, P.levels[acct], h->lev[acct].work);
    acct = -1;
  };
  for (int li = 0;; ++li) {
    sgf::Level& L = P.levels[li];
    LevelDev& D = h->lev[li];
    T* arena = D.arena.as<T>();
    T* blocks = arena + L.front_elems;
    for (const auto& el : L.elim) {
      h->max_m_all = std::max(h->max_m_all, el.m);
      h->max_k_all = std::max(h->max_k_all, el.k);
    }
    h->max_t = std::max(h->max_t, L.t_elems);
    double lvl_elim_flops = 0, lvl_elim_bytes = 0;
    for (const auto& d : L.elim) {
      lvl_elim_flops += elim_flops(d.m, d.k, d.bw);
      lvl_elim_bytes += elim_bytes(d.m, d.k, d.bw, sizeof(T));
    }
    if (L.top) {
      factor_top<T>(h, L, D, st);
    } else if (D.tiled) {
      D.banded_w = 0;
      tiled_factor<T>(h, st, D.h_tf, D.tf.as<sgf::TFront>(), arena, D.zt.as<T>(), L.t, "elim");
    } else if ((D.banded_w = banded_w(h, L, D)) > 0) {
      // one launch per ring-width class: the class with the most fronts on
      // the caller's stream, the others (typically a few boundary fronts with
      // a wider band, whose latency would otherwise add up) on the side
      // stream at the same time; timed as one launch
      int main_c = 0;
      for (int c = 1; c < 4; ++c)
        if (D.band_ptr[c + 1] - D.band_ptr[c] > D.band_ptr[main_c + 1] - D.band_ptr[main_c]) main_c = c;
      auto go = [&](int c, hipStream_t s) {
        const unsigned cnt = (unsigned)(D.band_ptr[c + 1] - D.band_ptr[c]);
        const int w = 8 * (c + 1);
        const size_t lds = (size_t)sgf::elim_banded_lds_elems(w) * sizeof(T);
        const int32_t* lst = D.band_list.as<int32_t>() + D.band_ptr[c];
        const sgf::ElimDesc* dd = D.elim.as<sgf::ElimDesc>();
        int* fl = h->d_fail.as<int>();
        T* pkp = D.pk.as<T>();
        switch (w) {
          case 8: hipLaunchKernelGGL((sgf::k_elim_banded<T, 8>), dim3(cnt), dim3(sgf::WAVE), lds, s, dd, arena, fl, lst, pkp); break;
          case 16: hipLaunchKernelGGL((sgf::k_elim_banded<T, 16>), dim3(cnt), dim3(sgf::WAVE), lds, s, dd, arena, fl, lst, pkp); break;
          case 24: hipLaunchKernelGGL((sgf::k_elim_banded<T, 24>), dim3(cnt), dim3(sgf::WAVE), lds, s, dd, arena, fl, lst, pkp); break;
          default: hipLaunchKernelGGL((sgf::k_elim_banded<T, 32>), dim3(cnt), dim3(sgf::WAVE), lds, s, dd, arena, fl, lst, pkp); break;
        }
      };
      D.pk.ensure((size_t)std::max<int64_t>(D.pk_elems, 1) * sizeof(T));
      // two classes (the common case: the fronts of a grid and its few wider
      // boundary blocks): one launch, the other class's fronts dispatched
      // first (k_elim_banded2)
      int other_c = -1, nclass = 0;
      for (int c = 0; c < 4; ++c)
        if (D.band_ptr[c + 1] > D.band_ptr[c]) {
          ++nclass;
          if (c != main_c) other_c = c;
        }
      const int wa = other_c >= 0 ? 8 * (other_c + 1) : 0, wb = 8 * (main_c + 1);
      const bool merged = nclass == 2 && ((wa == 24 && wb == 16) || (wa == 32 && wb == 16) || (wa == 16 && wb == 8));
      if (merged) {
        launch(h, st, "elim_banded", lvl_elim_flops, lvl_elim_bytes, [&] {
          const unsigned na = (unsigned)(D.band_ptr[other_c + 1] - D.band_ptr[other_c]);
          const unsigned nb = (unsigned)(D.band_ptr[main_c + 1] - D.band_ptr[main_c]);
          const size_t lds = (size_t)std::max(sgf::elim_banded_lds_elems(wa), sgf::elim_banded_lds_elems(wb)) * sizeof(T);
          const int32_t* la = D.band_list.as<int32_t>() + D.band_ptr[other_c];
          const int32_t* lb = D.band_list.as<int32_t>() + D.band_ptr[main_c];
          const sgf::ElimDesc* dd = D.elim.as<sgf::ElimDesc>();
          int* fl = h->d_fail.as<int>();
          T* pkp = D.pk.as<T>();
          if (wa == 24)
            hipLaunchKernelGGL((sgf::k_elim_banded2<T, 24, 16>), dim3(na + nb), dim3(sgf::WAVE), lds, st, dd, arena, fl,
                               la, (int)na, lb, pkp);
          else if (wa == 32)
            hipLaunchKernelGGL((sgf::k_elim_banded2<T, 32, 16>), dim3(na + nb), dim3(sgf::WAVE), lds, st, dd, arena, fl,
                               la, (int)na, lb, pkp);
          else
            hipLaunchKernelGGL((sgf::k_elim_banded2<T, 16, 8>), dim3(na + nb), dim3(sgf::WAVE), lds, st, dd, arena, fl,
                               la, (int)na, lb, pkp);
        }, L.t);
      } else
      launch(h, st, "elim_banded", lvl_elim_flops, lvl_elim_bytes, [&] {
        bool forked = false;
        for (int c = 0; c < 4; ++c) {
          if (c == main_c || D.band_ptr[c + 1] == D.band_ptr[c]) continue;
          if (!forked) {
            if (!h->side_stream) HIP_CHECK(hipStreamCreateWithFlags(&h->side_stream, hipStreamNonBlocking));
            if (!h->ev_fork) HIP_CHECK(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
            if (!h->ev_join) HIP_CHECK(hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming));
            HIP_CHECK(hipEventRecord(h->ev_fork, st));
            HIP_CHECK(hipStreamWaitEvent(h->side_stream, h->ev_fork, 0));
            forked = true;
          }
          go(c, h->side_stream);
        }
        go(main_c, st);
        if (forked) {
          HIP_CHECK(hipEventRecord(h->ev_join, h->side_stream));
          HIP_CHECK(hipStreamWaitEvent(st, h->ev_join, 0));
        }
      }, L.t);
      if (li == 0) D.front_clean = true;
    } else if (!L.elim.empty()) {
      int max_m = 0;
      for (const auto& e : L.elim) max_m = std::max(max_m, e.m);
      int nb = level_nb(h, L, max_m);
      size_t lds = (size_t)sgf::potrf_lds_elems(L.max_front_rows, nb) * sizeof(T);
      const int ne = (int)L.elim.size();
      bool persist = false;
      const unsigned grid = work_grid(ne, &persist, h->persist_cap);
      if (persist) HIP_CHECK(hipMemsetAsync(h->d_ctr.p, 0, sizeof(int), st));
      launch(h, st, "elim", lvl_elim_flops, lvl_elim_bytes, [&] {
        launch_elim<T>(nb, grid, lds, st, D.elim.as<sgf::ElimDesc>(), arena, h->d_fail.as<int>(),
                       D.elim_order.as<int32_t>(), ne,
                       persist ? h->d_ctr.as<int>() : nullptr);
      }, L.t);
    }
    h->trace.mark("elimination queued", L.t);
    if (L.top) {
      account_pending();
      int f = check_fail(h, st);
      HIP_CHECK(hipGetLastError());
      if (f >= 0) {
        h->failed_cluster = f;
        h->failed_level = L.t;
        throw SgfError(SGF_ENOTSPD, "non-positive pivot at the top node");
      }
      account_level(h, L, D.work);
      break;
    }
    if (!L.pairs.empty()) {
      double sb = 0;
      for (const auto& p : L.pairs) sb += (double)p.s_a * p.s_b * (p.c_cnt + 2) * e;
      launch(h, st, "schur", 0, sb, [&] {
        hipLaunchKernelGGL(sgf::k_schur<T>, dim3((unsigned)L.pairs.size()), dim3(sgf::WG), 0, st,
                           D.pairs.as<sgf::PairDesc>(), D.schur.as<sgf::SchurDesc>(), arena, blocks);
      }, L.t);
    }
    const int32_t* fixed = nullptr;
    if (!L.comp.empty() && h->low_rank) {
      if (li >= (int)h->lr_rank.size() || h->lr_rank[li].size() != L.comp.size())
        throw SgfError(SGF_ESTATE, "low-rank mode: the recorded ranks do not match level " + std::to_string(L.t));
      BatchScope bs(h);
      upload(h, D.fixrank, h->lr_rank[li], st);
      bs.flush(st);
      fixed = D.fixrank.as<int32_t>();
    }
    if (!L.comp.empty()) {
      // N in LDS when the widest one fits beside its column norms
      int64_t n_lds = 0;
      for (const auto& d : L.comp) n_lds = std::max<int64_t>(n_lds, (int64_t)d.s * d.c + ((d.c + 3) & ~3));
      const bool nlds = (size_t)n_lds * sizeof(T) <= LDS_BYTES;
      const int64_t extra = nlds ? n_lds : L.max_c;
      int nb = 4;
      size_t lds = (size_t)extra * sizeof(T);
      // small separators: one wavefront each, everything in LDS
      int snb = 0;
      size_t slds = 0;
      if (h->small_comp && h->persist_cap == 0) {
        int ms = 0, mc = 0;
        int64_t el = 0;
        for (const auto& d : L.comp) {
          ms = std::max(ms, d.s);
          mc = std::max(mc, d.c);
          el = std::max(el, sgf::comp_small_lds_elems(d.s, d.K, d.c, P.pi));
        }
        slds = (size_t)el * sizeof(T);
        if (ms <= sgf::CS_SMAX && mc <= sgf::CS_CMAX && slds <= LDS_BYTES) snb = ms <= 16 ? 16 : ms <= 32 ? 32 : 64;
      }
      // compression fronts [M_BB ; M_XB] gathered from the pair blocks, here
      // or (one-wavefront compressions of unfactored fronts) inside the
      // compression kernel
      const bool gather_inside = snb > 0 && !D.comp_tiled;
      if (!gather_inside)
        launch(h, st, "comp_gather", 0, 2.0 * L.cf_elems * e, [&] {
          hipLaunchKernelGGL(sgf::k_comp_gather<T>, dim3((unsigned)L.comp.size()), dim3(sgf::WG), 0, st,
                             D.comp.as<sgf::CompDesc>(), D.compnbr.as<sgf::CompNbr>(), blocks, D.cf.as<T>());
        }, L.t);
      if (D.comp_tiled) {
        // L_B and L_B^{-1} M_BX of every front by the tiled kernels first
        tiled_factor<T>(h, st, D.h_ctf, D.ctf.as<sgf::TFront>(), D.cf.as<T>(), nullptr, L.t, "comp", false);
      } else if (!snb) {
        nb = nb_for(L.max_cf_rows, L.max_s, sizeof(T), extra);
        lds = std::max<size_t>(sgf::potrf_lds_elems(L.max_cf_rows, nb), (size_t)extra) * sizeof(T);
      }
      if (lds > LDS_BYTES) throw SgfError(SGF_EINVAL, "compression kernel needs more LDS than available");
      double tol = P.opt.rank_tol;
      const int pre = D.comp_tiled ? 1 : 0;
      D.comp_small = snb > 0;
      if (snb) {
        const int bf = P.opt.precision == SGF_FP32_BF16N ? 1 : 0;
        D.tb.ensure((size_t)std::max<int64_t>(L.tb_elems, 1) * sizeof(T));
        launch(h, st, "compress", 0, 0, [&] {
          const dim3 g((unsigned)L.comp.size());
          auto a = std::make_tuple(D.comp.as<sgf::CompDesc>(), D.compnbr.as<sgf::CompNbr>(), D.cf.as<T>(),
                                   D.nbuf.as<T>(), (const T*)D.phi.as<T>(), D.ltphi.as<T>(), D.tau.as<T>(),
                                   D.rank.as<int>(), P.pi, tol, h->d_fail.as<int>(), pre, bf, D.tb.as<T>(),
                                   gather_inside ? (const T*)blocks : (const T*)nullptr, fixed);
          // few separators: four wavefronts each (the parallel phases spread
          // over them); many: one each, so that more separators share the chip
          // (measured on the 1024^2 grid: 480 separators and fewer gain, 1984 lose)
          const bool wide = !h->small_comp_one && L.comp.size() < 1024 && snb <= 32;
          const dim3 b1(sgf::WAVE), b4(4 * sgf::WAVE);
          std::apply([&](auto... x) {
            if (snb == 16 && wide) hipLaunchKernelGGL((sgf::k_compress_small<T, 16, 4>), g, b4, slds, st, x...);
            else if (snb == 16) hipLaunchKernelGGL((sgf::k_compress_small<T, 16, 1>), g, b1, slds, st, x...);
            else if (snb == 32 && wide) hipLaunchKernelGGL((sgf::k_compress_small<T, 32, 4>), g, b4, slds, st, x...);
            else if (snb == 32) hipLaunchKernelGGL((sgf::k_compress_small<T, 32, 1>), g, b1, slds, st, x...);
            else hipLaunchKernelGGL((sgf::k_compress_small<T, 64, 1>), g, b1, slds, st, x...);
          }, a);
        }, L.t);
      }
      bool cpersist = false;
      const unsigned cgrid = work_grid((int)L.comp.size(), &cpersist, h->persist_cap);
      if (cpersist) HIP_CHECK(hipMemsetAsync(h->d_ctr.p, 0, sizeof(int), st));
      if (!snb) launch(h, st, "compress", 0, 0, [&] {
        launch_compress<T>(nlds, cpersist, nb, cgrid, lds, st, D.comp.as<sgf::CompDesc>(),
                           D.compnbr.as<sgf::CompNbr>(), D.cf.as<T>(), D.nbuf.as<T>(), D.phi.as<T>(), D.ltphi.as<T>(),
                           D.tau.as<T>(), D.rank.as<int>(), P.pi, tol, h->d_fail.as<int>(), pre,
                           P.opt.precision == SGF_FP32_BF16N ? 1 : 0, D.comp_order.as<int32_t>(), (int)L.comp.size(),
                           cpersist ? h->d_ctr.as<int>() : nullptr, fixed);
      }, L.t);
      launch(h, st, "phi_commit", 0, 0, [&] {
        hipLaunchKernelGGL(sgf::k_phi_commit<T>, dim3((unsigned)L.comp.size()), dim3(sgf::WG), 0, st,
                           D.comp.as<sgf::CompDesc>(), D.rank.as<int>(), D.ltphi.as<T>(), D.phi.as<T>(), P.pi);
      }, L.t);
    }
    HIP_CHECK(hipGetLastError());
    L.rank.assign(L.comp.size(), 0);
    if (!L.comp.empty())
      HIP_CHECK(hipMemcpyAsync(L.rank.data(), D.rank.p, L.comp.size() * sizeof(int), hipMemcpyDeviceToHost, st));
    const bool reuse_next = (int)P.levels.size() > li + 1 && (int)h->lev.size() > li + 1 &&
                            h->lev[li + 1].uploaded;
    account_pending();
    int f = check_fail(h, st);
    if (f >= 0) {
      h->failed_cluster = f;
      h->failed_level = L.t;
      throw SgfError(SGF_ENOTSPD, "non-positive pivot at level " + std::to_string(L.t));
    }
    h->trace.mark("synchronized (ranks read)", L.t);
    if (h->prof.on && !L.comp.empty()) {
      double cf = 0, cb = 0;
      for (size_t c = 0; c < L.comp.size(); ++c) {
        const auto& d = L.comp[c];
        cf += comp_flops(d.s, d.K, d.c, L.rank[c], P.pi, D.comp_tiled);
        cb += comp_bytes(d.s, d.K, d.c, L.rank[c], P.pi, D.comp_tiled, sizeof(T));
      }
      h->prof.charge("compress", L.t, cf, cb);
    }
    const bool same_ranks = reuse_next && L.rank == L.planned_rank;
    if (h->trace.on) {
      int ndiff = -1;
      if (L.rank.size() == L.planned_rank.size()) {
        ndiff = 0;
        for (size_t c = 0; c < L.rank.size(); ++c) ndiff += L.rank[c] != L.planned_rank[c];
      }
      std::fprintf(stderr, "[sgf] level %d: reuse_next %d, ranks %zu, planned %zu, differing %d\n", L.t,
                   (int)reuse_next, L.rank.size(), L.planned_rank.size(), ndiff);
    }
    const bool emit = !h->device_coarsen;
    if (!same_ranks) {
      for (size_t q = li + 1; q < h->lev.size(); ++q) h->lev[q].uploaded = false;
      P.max_node = 0;
      for (int q = 0; q <= li; ++q)
        for (int sz : P.levels[q].size) P.max_node = std::max<int64_t>(P.max_node, sz);
    }
    auto comp_work = [&] {
      // compressed separators of this level, for the apply
      L.capply.clear();
      std::vector<int64_t> cap_tb;   // T_B slot of each compressed separator (small compressions)
      for (size_t c = 0; c < L.comp.size(); ++c) {
        const auto& d = L.comp[c];
        if (L.rank[c] < d.s) {
          cap_tb.push_back(d.tb_off);
          sgf::CompApply a{};
          a.cf_off = d.cf_off;
          a.v_off = d.n_off;
          a.tau_off = d.tau_off;
          a.slot_off = d.slot_off;
          a.s = d.s;
          a.ld = d.s + d.K;
          a.r = L.rank[c];
          L.capply.push_back(a);
          h->max_s_all = std::max(h->max_s_all, d.s);
          ++h->compressed;
        }
      }
      {
        // T_B slots: the planned ones when the small compression formed T_B,
        // else packed over the compressed separators for k_comp_explicit
        int64_t toff = 0, voff = 0;
        for (size_t q = 0; q < L.capply.size(); ++q) {
          auto& a = L.capply[q];
          a.t_off = D.comp_small ? cap_tb[q] : toff;
          toff += (int64_t)a.s * a.s;
          a.v_off2 = (int32_t)voff;
          voff += a.s;
        }
        D.tb.ensure(std::max<int64_t>(D.comp_small ? L.tb_elems : toff, 1) * sizeof(T));
        D.c_elems = voff;
      }
      {
        BatchScope bs(h);
        if (!same_ranks || D.capply_small != D.comp_small) {
          D.capply_small = D.comp_small;
          upload(h, D.capply, L.capply, st);
          L.t_of_comp.assign(L.comp.size(), -1);
          std::vector<int32_t> q_of_comp(L.comp.size(), -1);
          for (size_t c = 0, q = 0; c < L.comp.size(); ++c)
            if (L.rank[c] < L.comp[c].s) {
              q_of_comp[c] = (int32_t)q;
              L.t_of_comp[c] = L.capply[q++].t_off;
            }
          upload(h, D.tofcomp, L.t_of_comp, st);
          // compressed separator of every accumulation entry (for the fused
          // forward separator step)
          L.cap_of_acc.assign(L.sepacc.size(), -1);
          size_t covered = 0;
          for (size_t a = 0; a < L.sepacc.size(); ++a) {
            const int c = L.comp_of[L.seps[L.sacc_p[a]]];
            if (c >= 0 && q_of_comp[c] >= 0) {
              L.cap_of_acc[a] = q_of_comp[c];
              ++covered;
            }
          }
          L.acc_covers_capply = covered == L.capply.size();
          upload(h, D.capacc, L.cap_of_acc, st);
        }
        // pairs that touch a compressed separator (their coarse couplings)
        if (!L.capply.empty() && !same_ranks) {
          L.active_pairs.clear();
          for (size_t p = 0; p < L.pairs.size(); ++p) {
            const auto& pd = L.pairs[p];
            const bool ca = pd.ca >= 0 && L.rank[pd.ca] < pd.s_a, cb = pd.cb >= 0 && L.rank[pd.cb] < pd.s_b;
            if (ca || cb) L.active_pairs.push_back((int32_t)p);
          }
          upload(h, D.active, L.active_pairs, st);
        }
        bs.flush(st);
      }
      if (!L.capply.empty() && !D.comp_small) {
        double fl = 0;
        for (auto& a : L.capply) fl += (double)a.s * a.s * a.s / 3.0 + 4.0 * a.s * a.s * a.r;
        launch(h, st, "comp_explicit", fl, 0, [&] {
          int smax = 0;
          for (auto& a : L.capply) smax = std::max(smax, a.s);
          hipLaunchKernelGGL(sgf::k_comp_explicit<T>, dim3((unsigned)L.capply.size(), cdiv(smax, sgf::CEB)),
                             dim3(sgf::WG), 0, st,
                             D.capply.as<sgf::CompApply>(), D.cf.as<T>(), D.nbuf.as<T>(), D.tau.as<T>(), D.tb.as<T>());
        }, L.t);
      }
      // coarse couplings, only for the pairs that touch a compressed separator
      if (!L.capply.empty()) {
        // many small pairs: one wavefront each, T_a M_ab in LDS
        int64_t gmax = 1;
        for (int32_t p : L.active_pairs) {
          const auto& pd = L.pairs[p];
          const int ra = pd.ca >= 0 && L.rank[pd.ca] < pd.s_a ? L.rank[pd.ca] : pd.s_a;
          gmax = std::max<int64_t>(gmax, (int64_t)ra * pd.s_b);
        }
        const size_t plds = (size_t)sgf::PPB * gmax * sizeof(T);
        const unsigned nact = (unsigned)L.active_pairs.size();
        launch(h, st, "pair", 0, 0, [&] {
          const bool wave = plds <= LDS_BYTES && (h->pair_mode == 1 || (h->pair_mode < 0 && nact >= 4096));
          if (wave)
            hipLaunchKernelGGL(sgf::k_pair_w<T>, dim3(cdiv(nact, sgf::PPB)), dim3(sgf::PPB * sgf::WAVE), plds, st,
                               D.pairs.as<sgf::PairDesc>(), D.active.as<int32_t>(), (int)nact, D.rank.as<int>(),
                               D.tofcomp.as<int64_t>(), D.tb.as<T>(), blocks, (int)gmax);
          else
            hipLaunchKernelGGL(sgf::k_pair<T>, dim3(nact), dim3(sgf::WG), 0, st, D.pairs.as<sgf::PairDesc>(),
                               D.active.as<int32_t>(), D.rank.as<int>(), D.tofcomp.as<int64_t>(), D.tb.as<T>(), blocks,
                               D.scratch.as<T>());
        }, L.t);
      }
      acct = li;   // counted while the GPU runs the next level
    };
    // The next level's in-place re-plan for these ranks (its structure does
    // not depend on them: only sizes and offsets are redone) reads only this
    // level's ranks and the plan; the compressed-separator work above reads
    // and writes other fields of this level and queues device work.  So the
    // worker thread queues that work while this thread, whose caches hold
    // the plan, re-plans; the worker is joined before anything else (or on
    // the way out of an error).
    // (only on large levels: on small ones waking the worker costs more than
    // the overlap saves, 10-20 us per level measured)
    bool planned = false;
    if (!same_ranks && L.pairs.size() >= 2048 && sgf::can_update_next_level(P, (size_t)li)) {
      h->worker.start(comp_work);
      WorkerJoin wjoin{&h->worker, true};
      planned = sgf::update_next_level(P, (size_t)li, D.h_blkmap, D.h_phimap, emit);
      wjoin.active = false;
      h->worker.wait();
    } else {
      comp_work();
      if (!same_ranks) planned = sgf::update_next_level(P, (size_t)li, D.h_blkmap, D.h_phimap, emit);
    }
    h->trace.mark("compressed-separator work queued", L.t);
    // ---- coarsen (Secs. 4.3-4.4) ----------------------------------------------
    {
      BatchScope bs(h);
      if (!same_ranks) {
        // the in-place re-plan, else a fresh one
        bool fresh = false;
        if (!planned) {
          P.levels.resize(li + 1);
          P.parts.resize(li + 1);
          sgf::plan_next_level(P, D.h_blkmap, D.h_phimap, emit);
          fresh = true;
        }
        h->trace.mark("next level planned (host)", li + 1);
        if (emit) {
          upload(h, D.blkmap, D.h_blkmap, st);
          upload(h, D.phimap, D.h_phimap, st);
        } else {
          sgf::Level& Cl = P.levels[li];
          sgf::Level& Nl = P.levels[li + 1];
          if (fresh || !D.coarsen_static) {
            sgf::coarsen_tables(Cl, Nl, D.h_cpairs, D.h_cseps);
            upload(h, D.cpairs, D.h_cpairs, st);
            upload(h, D.cseps, D.h_cseps, st);
            D.coarsen_static = true;
          }
          upload(h, D.cfather, Nl.cp_father, st);
          upload(h, D.cloc, Nl.cp_loc, st);
        }
      }
      upload_level(h, li + 1, st);
      h->trace.mark("next level tables built (host)", li + 1);
      bs.flush(st);
    }
    h->trace.mark(same_ranks ? "next level reused" : "next level uploaded", li + 1);
    sgf::Level& N = P.levels[li + 1];
    LevelDev& E = h->lev[li + 1];
    LevelDev& Dc = h->lev[li];   // re-fetch: lev may have grown
    const int64_t ne = N.front_elems + N.blk_elems;
    launch(h, st, "zero", 0, ne * e, [&] { zero<T>(E.arena, ne, st); });
    // pair blocks and Phi rows of the surviving separators into the new
    // level, one launch for both
    if (h->device_coarsen) {
      // re-fetch: planning the next level may have reallocated P.levels
      const sgf::Level& C = P.levels[li];
      const unsigned np = (unsigned)C.pairs.size(), ns = (unsigned)C.seps.size();
      // the tables the kernel indexes must hold its grid's items
      if (Dc.pairs.bytes < np * sizeof(sgf::PairDesc) || Dc.cpairs.bytes < np * sizeof(sgf::CoarsenPair) ||
          Dc.cseps.bytes < ns * sizeof(sgf::CoarsenSep) || Dc.cfather.bytes < ns * sizeof(int32_t) ||
          Dc.cloc.bytes < ns * sizeof(int32_t) || C.rank.size() != C.comp.size() ||
          N.cp_father.size() != ns || N.cp_loc.size() != ns ||
          E.nbroff.bytes < N.nbr_off.size() * sizeof(int32_t) ||
          E.elim.bytes < N.elim.size() * sizeof(sgf::ElimDesc) || E.pairs.bytes < N.pairs.size() * sizeof(sgf::PairDesc))
        throw SgfError(SGF_EINVAL, "coarsening tables do not match the level sizes");
      double cb = 0;
      if (h->prof.on)
        for (const auto& pd : C.pairs) {
          const int ra = pd.ca >= 0 && C.rank[pd.ca] < pd.s_a ? C.rank[pd.ca] : pd.s_a;
          const int rb = pd.cb >= 0 && C.rank[pd.cb] < pd.s_b ? C.rank[pd.cb] : pd.s_b;
          cb += (pd.a == pd.b ? 2.0 : 3.0) * ra * rb * e;
        }
      if (np + ns > 0)
        launch(h, st, "coarsen_copy", 0, cb, [&] {
          hipLaunchKernelGGL(sgf::k_coarsen<T>, dim3(np + ns), dim3(sgf::WG), 0, st, Dc.pairs.as<sgf::PairDesc>(),
                             Dc.cpairs.as<sgf::CoarsenPair>(), (int)np, Dc.cseps.as<sgf::CoarsenSep>(), (int)ns,
                             Dc.rank.as<int>(), Dc.cfather.as<int32_t>(), Dc.cloc.as<int32_t>(),
                             E.elim.as<sgf::ElimDesc>(), (int)N.elim.size(), E.pairs.as<sgf::PairDesc>(),
                             (int)N.pairs.size(), E.nbroff.as<int32_t>(), (int64_t)N.nbr_off.size(),
                             (int)N.cell.size(), (int)C.comp.size(),
                             (const T*)Dc.arena.as<T>(), C.front_elems, C.front_elems + C.blk_elems, E.arena.as<T>(),
                             N.front_elems, ne, Dc.slotptr.as<int64_t>(), Dc.phioff.as<int64_t>(),
                             (const T*)Dc.phi.as<T>(), C.phi_elems, E.slotptr.as<int64_t>(), E.phioff.as<int64_t>(),
                             E.phi.as<T>(), N.phi_elems, P.pi, N.top ? 0 : 1, h->d_fail.as<int>() + 1);
        }, li + 1);
    }
    const unsigned nbm = h->device_coarsen ? 0u : (unsigned)Dc.h_blkmap.size();
    const unsigned npm = h->device_coarsen ? 0u : (unsigned)Dc.h_phimap.size();
    if (nbm + npm > 0) {
      double cb = 0;
      if (h->prof.on)
        for (const auto& c : Dc.h_blkmap) cb += 2.0 * c.rows * c.cols * e;
      launch(h, st, "coarsen_copy", 0, cb, [&] {
        hipLaunchKernelGGL(sgf::k_copy_blocks2<T>, dim3(nbm + npm), dim3(sgf::WG), 0, st,
                           Dc.blkmap.as<sgf::CopyDesc>(), (const T*)Dc.arena.as<T>(), E.arena.as<T>(), (int)nbm,
                           Dc.phimap.as<sgf::CopyDesc>(), (const T*)Dc.phi.as<T>(), E.phi.as<T>());
      }, li + 1);
    }
    HIP_CHECK(hipGetLastError());
    h->trace.mark("coarsening queued", li + 1);
  }
  h->trace.mark("done", (int)P.levels.size());
  // device bytes held by the factor
  h->factor_bytes = 0;
  for (size_t li = 0; li < P.levels.size(); ++li) {
    const auto& D = h->lev[li];
    h->factor_bytes += D.arena.bytes + D.cf.bytes + D.nbuf.bytes + D.tau.bytes + D.tb.bytes;
    if (D.tiled) h->factor_bytes += D.zt.bytes;
  }
  h->factor_bytes += h->top64.bytes + (h->top_tiled ? h->topz.bytes : 0);
  const auto& top = P.levels.back().elim[0];
  h->max_m_all = std::max(h->max_m_all, top.m);
  int64_t n = P.n;
  h->apply_bytes += 2.0 * n * (8 + e + 8);  // permutation gather / scatter
  h->factored = true;
}

// Work vectors of one apply: the permuted vector y (n per column), the
// separator scratch (max_t per column), and per level the compressed
// separators' vector (tiled path) and the tiled fronts' work vector, and the
// top's (FP64).  Normally the handle's own buffers; the allocation-free
// apply carves them out of the library's static device scratch.
struct ApplyWork {
  static constexpr int MAXL = 64;
  void* y = nullptr;
  void* tscr = nullptr;
  void* topu = nullptr;
  void* cw[MAXL] = {};
  void* uw[MAXL] = {};
};

ApplyWork handle_work(sgf_handle h) {
  ApplyWork w;
  w.y = h->y.p;
  w.tscr = h->tscr.p;
  w.topu = h->topu.p;
  for (size_t li = 0; li < h->lev.size() && li < (size_t)ApplyWork::MAXL; ++li) {
    w.cw[li] = h->lev[li].cw.p;
    w.uw[li] = h->lev[li].uw.p;
  }
  return w;
}

// Work vectors of the apply for nrhs columns.  A captured apply or PCG
// graph holds the addresses of these buffers, so when one of them is
// reallocated (grown) the epoch advances and every graph recorded before is
// captured anew instead of replayed on freed memory.
template <typename T>
void ensure_work(sgf_handle h, int nrhs) {
  std::vector<const void*> before, after;
  auto addrs = [&](std::vector<const void*>& v) {
    v.clear();
    v.push_back(h->y.p);
    v.push_back(h->tscr.p);
    v.push_back(h->topu.p);
    for (auto& D : h->lev) {
      v.push_back(D.uw.p);
      v.push_back(D.cw.p);
    }
  };
  addrs(before);
  h->y.ensure((size_t)h->plan.n * nrhs * sizeof(T));
  for (auto& D : h->lev) {
    if (D.tiled && D.uploaded) D.uw.ensure((size_t)std::max<int64_t>(D.u_elems, 1) * nrhs * sizeof(T));
    if (D.uploaded) D.cw.ensure((size_t)std::max<int64_t>(D.c_elems, 1) * nrhs * sizeof(T));
  }
  if (h->top_tiled) h->topu.ensure((size_t)h->top_R * nrhs * sizeof(double));
  h->tscr.ensure((size_t)std::max<int64_t>(h->max_t, 1) * nrhs * sizeof(T));
  addrs(after);
  if (before != after) ++h->epoch;
}

void ensure_work_any(sgf_handle h, int nrhs) {
  if (h->esz == 8) ensure_work<double>(h, nrhs);
  else ensure_work<float>(h, nrhs);
}

// Right-hand sides per workgroup of an apply kernel whose LDS holds `fixed`
// bytes plus `per_rhs` bytes per column.
int rc_for(size_t fixed, size_t per_rhs, int nrhs) {
  if (fixed + per_rhs > LDS_BYTES) throw SgfError(SGF_EINVAL, "apply kernel needs more LDS than available");
  int rc = std::min(sgf::RCM, nrhs);
  while (rc > 1 && fixed + rc * per_rhs > LDS_BYTES) --rc;
  return rc;
}

template <typename T, bool PK, typename... A>
void band_fwd_launch(int rc, dim3 g, size_t lds, hipStream_t st, A... a) {
  if (rc == 1) hipLaunchKernelGGL((sgf::k_band_fwd<T, 1, PK>), g, dim3(sgf::WG), lds, st, a...);
  else if (rc == 2) hipLaunchKernelGGL((sgf::k_band_fwd<T, 2, PK>), g, dim3(sgf::WG), lds, st, a...);
  else if (rc == 3) hipLaunchKernelGGL((sgf::k_band_fwd<T, 3, PK>), g, dim3(sgf::WG), lds, st, a...);
  else hipLaunchKernelGGL((sgf::k_band_fwd<T, 4, PK>), g, dim3(sgf::WG), lds, st, a...);
}
template <typename T, bool PK, typename... A>
void band_bwd_launch(int rc, dim3 g, size_t lds, hipStream_t st, A... a) {
  if (rc == 1) hipLaunchKernelGGL((sgf::k_band_bwd<T, 1, PK>), g, dim3(sgf::WG), lds, st, a...);
  else if (rc == 2) hipLaunchKernelGGL((sgf::k_band_bwd<T, 2, PK>), g, dim3(sgf::WG), lds, st, a...);
  else if (rc == 3) hipLaunchKernelGGL((sgf::k_band_bwd<T, 3, PK>), g, dim3(sgf::WG), lds, st, a...);
  else hipLaunchKernelGGL((sgf::k_band_bwd<T, 4, PK>), g, dim3(sgf::WG), lds, st, a...);
}

// Whether the interior sweeps of a level run the banded kernels: enabled,
// one-workgroup fronts, a band of at most BAND_MAX and the LDS for one rhs.
// Columns per transposed L_SI tile of the banded backward sweep: 64, halved
// while one right-hand side's LDS does not fit (at least 8).
int band_tj(sgf_handle h, const LevelDev& D) {
  int tj = sgf::WAVE;
  while (tj > 8 && (size_t)sgf::band_bwd_lds(D.band_m, D.band_k, D.band_bw, 1, tj) * h->esz > LDS_BYTES) tj /= 2;
  return tj;
}
int64_t band_lds(sgf_handle h, const LevelDev& D, bool fwd, int rc) {
  return fwd ? sgf::band_fwd_lds(D.band_m, D.band_k, D.band_bw, rc)
             : sgf::band_bwd_lds(D.band_m, D.band_k, D.band_bw, rc, band_tj(h, D));
}
// Banded sweeps for levels whose fronts are banded (the widest band below
// the largest front's size - 1, or the banded elimination's packed copy):
// on dense upper-level fronts the blocked sweeps measured faster.
bool band_level(sgf_handle h, const LevelDev& D, bool fwd) {
  if (!h->band_apply || D.tiled || D.band_bw < 0 || D.band_bw > sgf::BAND_MAX) return false;
  if (D.banded_w == 0 && D.band_bw >= D.band_m - 1) return false;
  return (size_t)band_lds(h, D, fwd, 1) * h->esz <= LDS_BYTES;
}
// One right-hand side on a level eliminated by the banded kernel (packed
// copy present): band solves one wavefront per front and the L_SI products
// one workgroup per front (k_band1_solve, k_band1_lsi, k_band1_lsit) when
// enabled and their LDS fits.  *nb: band rows staged (16 or 32), *per_wave:
// LDS elements per wavefront of the solves.
// Fronts (wavefronts) per workgroup of the band solves staging nb band rows:
// of 1, 2 and 4 (within the workgroup LDS limit), the one that keeps the
// most wavefronts resident in a compute unit's 160 KiB of LDS (counted up to
// 16, what their registers allow), the larger on a tie.
int band1_fronts(sgf_handle h, const LevelDev& D, int nb) {
  constexpr size_t CU_LDS = 160 * 1024;
  const size_t per = (size_t)sgf::band1_lds_elems(D.band_m, nb) * h->esz;
  int best = 1;
  size_t best_waves = 0;
  for (int f = 1; f <= sgf::B1_FRONTS; f *= 2) {
    if ((size_t)f * per > LDS_BYTES) break;
    const size_t waves = std::min<size_t>((size_t)f * (CU_LDS / ((size_t)f * per)), 16);
    if (waves >= best_waves) best = f, best_waves = waves;
  }
  return best;
}
bool band1_level(sgf_handle h, const LevelDev& D, int nrhs, int* nb, int* per_wave) {
  if (nrhs != 1 || !h->band1 || D.banded_w <= 0 || !D.band_ok || D.band_k > sgf::BE_KMAX || D.band_bw > 31 ||
      D.band_m > sgf::B1_MAXC * sgf::WAVE)
    return false;
  *nb = 32;   // the widest class
  *per_wave = 0;
  const size_t solve = (size_t)sgf::band1_lds_elems(D.band_m, *nb) * h->esz;
  const size_t lsi = ((size_t)sgf::band1_xs(D.band_m) + 4 * sgf::WAVE) * h->esz;
  const size_t lsit = ((size_t)sgf::WAVE * (sgf::BE_KMAX | 1) + sgf::BE_KMAX + 4 * sgf::WAVE) * h->esz;
  return std::max(solve, std::max(lsi, lsit)) <= LDS_BYTES;
}

// Launches of the one-right-hand-side banded sweeps of level L (see
// band1_level): forward = band solve then t = L_SI x; backward = y_I -
// L_SI^T y_S then the transposed band solve.  Bytes charged: the band and the
// vectors to the solves, L_SI and its vectors to the products.
template <typename T>
void band1_sweep(sgf_handle h, const sgf::Level& L, LevelDev& D, bool fwd, int nb, int per_wave, T* y, T* ts,
                 hipStream_t st) {
  const int nf = (int)L.elim.size();
  const double e = sizeof(T);
  double band_b = 0, lsi_b = 0;
  for (const auto& el : L.elim) {
    const double m = el.m, k = el.k, bw = std::min(el.bw, std::max(el.m - 1, 0));
    band_b += (bw + 1) * m * e + 2 * m * e + 4 * m;
    lsi_b += k * m * e + (fwd ? m * e + 4 * m + k * e : 2 * m * e + 4 * m + k * (e + 4));
  }
  const sgf::ElimDesc* dd = D.elim.as<sgf::ElimDesc>();
  const int32_t* sl = D.slots.as<int32_t>();
  const T* pk = D.pk.as<T>();
  (void)per_wave;
  // fronts of bandwidth up to 16 stage 17 band rows, the others 32; one
  // launch per group, fronts per workgroup as band1_fronts chooses
  auto solve = [&] {
    launch(h, st, fwd ? "apply_band_fwd" : "apply_band_bwd", 0, band_b, [&] {
      const int32_t* bl = D.b1_list.as<int32_t>();
      const int n17 = D.b1_split, n32 = (int)D.h_b1_list.size() - D.b1_split;
      if (n17 > 0) {
        const int fw = band1_fronts(h, D, 17), pw = (int)sgf::band1_lds_elems(D.band_m, 17);
        const dim3 g(cdiv(n17, fw)), b(fw * sgf::WAVE);
        const size_t l = (size_t)fw * pw * sizeof(T);
        if (fwd) hipLaunchKernelGGL((sgf::k_band1_solve<T, 17, true>), g, b, l, st, dd, bl, n17, sl, y, pk, pw);
        else hipLaunchKernelGGL((sgf::k_band1_solve<T, 17, false>), g, b, l, st, dd, bl, n17, sl, y, pk, pw);
      }
      if (n32 > 0) {
        const int fw = band1_fronts(h, D, 32), pw = (int)sgf::band1_lds_elems(D.band_m, 32);
        const dim3 g(cdiv(n32, fw)), b(fw * sgf::WAVE);
        const size_t l = (size_t)fw * pw * sizeof(T);
        const int32_t* b2 = bl + D.b1_split;
        if (fwd) hipLaunchKernelGGL((sgf::k_band1_solve<T, 32, true>), g, b, l, st, dd, b2, n32, sl, y, pk, pw);
        else hipLaunchKernelGGL((sgf::k_band1_solve<T, 32, false>), g, b, l, st, dd, b2, n32, sl, y, pk, pw);
      }
    }, L.t);
  };
  if (fwd) {
    solve();
    const int xe = sgf::band1_xs(D.band_m);
    launch(h, st, "apply_lsi_fwd", 0, lsi_b, [&] {
      hipLaunchKernelGGL(sgf::k_band1_lsi<T>, dim3(nf), dim3(sgf::WG), (size_t)(xe + 4 * sgf::WAVE) * sizeof(T), st,
                         dd, sl, (const T*)y, ts, pk, xe);
    }, L.t);
  } else {
    launch(h, st, "apply_lsi_bwd", 0, lsi_b, [&] {
      hipLaunchKernelGGL(sgf::k_band1_lsit<T>, dim3(nf), dim3(sgf::WG),
                         ((size_t)sgf::WAVE * (sgf::BE_KMAX | 1) + sgf::BE_KMAX + 4 * sgf::WAVE) * sizeof(T), st, dd, sl,
                         D.nslots.as<int32_t>(), y, pk);
    }, L.t);
    solve();
  }
}
// Register rows of the small-separator paths of k_sepacc_comp and
// k_comp_apply_t for a level whose separators have at most s rows (0: the
// general path).
int small_rows(int s) { return s <= 16 ? 16 : s <= 32 ? 32 : s <= 64 ? 64 : 0; }

// One right-hand side on a level whose interiors all have at most 64 rows
// (k_apply1), when its LDS (the triangle tile and L_SI) fits and the level
// was not eliminated by the banded kernel (whose packed copy, read by the
// banded sweeps, holds the pivots' hardware reciprocals); *kmax: the level's
// largest k.
bool apply1_level(sgf_handle h, const sgf::Level& L, const LevelDev& D, int nrhs, int* kmax) {
  if (nrhs != 1 || !h->apply1 || L.elim.empty() || D.banded_w > 0) return false;
  int mm = 0, kk = 0;
  for (const auto& e : L.elim) {
    mm = std::max(mm, e.m);
    kk = std::max(kk, e.k);
  }
  *kmax = std::max(kk, 1);
  return mm <= sgf::WAVE && (size_t)sgf::apply1_lds_elems(*kmax) * h->esz <= LDS_BYTES;
}
// Right-hand sides per workgroup of the banded sweeps: at most one per
// wavefront and what the LDS holds.
int band_rc(sgf_handle h, const LevelDev& D, bool fwd, int nrhs) {
  int rc = std::min(sgf::RCM, nrhs);
  while (rc > 1 && (size_t)band_lds(h, D, fwd, rc) * h->esz > LDS_BYTES) --rc;
  return rc;
}

template <typename T>
void run_sweeps(sgf_handle h, int nrhs, bool product, hipStream_t st, const ApplyWork& W) {
  sgf::Plan& P = h->plan;
  const int64_t n = P.n;
  T* y = reinterpret_cast<T*>(W.y);
  T* ts = reinterpret_cast<T*>(W.tscr);
  const int64_t ldt = std::max<int64_t>(h->max_t, 1);
  const int nl = (int)P.levels.size();
  auto maxes = [](const sgf::Level& L, int& mm, int& mk, int& ms) {
    mm = mk = ms = 0;
    for (auto& e : L.elim) {
      mm = std::max(mm, e.m);
      mk = std::max(mk, e.k);
    }
    for (auto& a : L.capply) ms = std::max(ms, a.s);
  };
  auto elim_fwd = [&](int li, int mode) {
    sgf::Level& L = P.levels[li];
    LevelDev& D = h->lev[li];
    int mm, mk, ms;
    maxes(L, mm, mk, ms);
    if (L.elim.empty()) return;
    if (mode == 0 && D.tiled) {
      const unsigned nf = (unsigned)D.h_tf.size();
      const size_t e = sizeof(T), mp = (D.tmax_m + 3) & ~3;
      const int rc1 = rc_for(0, D.tmax_m * e, nrhs), rc2 = rc_for(0, (mp + sgf::WG) * e, nrhs);
      launch(h, st, "apply_elim_fwd", 0, 0.5 * (cdiv(nrhs, rc1) * D.work.fwd_bytes + nrhs * D.work.fwd_vec), [&] {
        hipLaunchKernelGGL((sgf::k_tfwd_z<T, T>), dim3(cdiv(D.tmax_m, sgf::TB), nf, cdiv(nrhs, rc1)), dim3(sgf::WG),
                           (size_t)rc1 * D.tmax_m * e, st, D.tf.as<sgf::TFront>(), D.zt.as<T>(),
                           D.slots.as<int32_t>(), y, n, reinterpret_cast<T*>(W.uw[li]), D.u_elems, nrhs, rc1);
      }, L.t);
      launch(h, st, "apply_elim_fwd", 0, 0.5 * (cdiv(nrhs, rc2) * D.work.fwd_bytes + nrhs * D.work.fwd_vec), [&] {
        hipLaunchKernelGGL((sgf::k_tfwd_s<T, T>), dim3(std::max(1u, cdiv(D.tmax_k, sgf::TB)), nf, cdiv(nrhs, rc2)),
                           dim3(sgf::WG), (size_t)rc2 * (mp + sgf::WG) * e, st, D.tf.as<sgf::TFront>(),
                           D.arena.as<T>(), reinterpret_cast<T*>(W.uw[li]), D.u_elems, D.slots.as<int32_t>(), y, n, ts, ldt, nrhs, rc2);
      }, L.t);
      return;
    }
    int nb1 = 0, pw = 0;
    if (mode == 0 && band_level(h, D, true) && band1_level(h, D, nrhs, &nb1, &pw)) {
      band1_sweep<T>(h, L, D, true, nb1, pw, y, ts, st);
      return;
    }
    int k1 = 0;
    if (mode == 0 && apply1_level(h, L, D, nrhs, &k1)) {
      const int order = band_level(h, D, true) ? 1 : 0;   // the summation order of the multi-column sweeps
      launch(h, st, "apply_small_fwd", 0, D.work.fwd_bytes + D.work.fwd_vec, [&] {
        hipLaunchKernelGGL((sgf::k_apply1<T, true>), dim3((unsigned)L.elim.size()), dim3(sgf::WG),
                           (size_t)sgf::apply1_lds_elems(k1) * sizeof(T), st, D.elim.as<sgf::ElimDesc>(),
                           (const T*)D.arena.as<T>(), D.slots.as<int32_t>(), D.nslots.as<int32_t>(), y, ts, k1, order);
      }, L.t);
      return;
    }
    if (mode == 0 && band_level(h, D, true)) {
      const int rc = band_rc(h, D, true, nrhs);
      const size_t lds = (size_t)sgf::band_fwd_lds(D.band_m, D.band_k, D.band_bw, rc) * sizeof(T);
      launch(h, st, "apply_band_fwd", 0, cdiv(nrhs, rc) * D.work.fwd_bytes + nrhs * D.work.fwd_vec, [&] {
        const dim3 g((unsigned)L.elim.size(), cdiv(nrhs, rc));
        const sgf::ElimDesc* dd = D.elim.as<sgf::ElimDesc>();
        const int32_t* sl = D.slots.as<int32_t>();
        if (D.banded_w > 0)
          band_fwd_launch<T, true>(rc, g, lds, st, dd, D.arena.as<T>(), sl, y, n, ts, ldt, nrhs, D.pk.as<T>());
        else
          band_fwd_launch<T, false>(rc, g, lds, st, dd, D.arena.as<T>(), sl, y, n, ts, ldt, nrhs, (const T*)nullptr);
      }, L.t);
      return;
    }
    if (mode == 0) {
      const size_t fixed = (size_t)sgf::DB * sgf::DLD * sizeof(T);
      const int rc = rc_for(fixed, (size_t)((L.max_front_rows + 3) & ~3) * sizeof(T), nrhs);
      const size_t lds = fixed + (size_t)rc * ((L.max_front_rows + 3) & ~3) * sizeof(T);
      launch(h, st, "apply_elim_fwd", 0, cdiv(nrhs, rc) * D.work.fwd_bytes + nrhs * D.work.fwd_vec, [&] {
        const dim3 g((unsigned)L.elim.size(), cdiv(nrhs, rc));
        const sgf::ElimDesc* dd = D.elim.as<sgf::ElimDesc>();
        const int32_t* sl = D.slots.as<int32_t>();
        if (rc == 1) hipLaunchKernelGGL((sgf::k_apply_fwd<T, 1>), g, dim3(sgf::WG), lds, st, dd, D.arena.as<T>(), sl, y, n, ts, ldt, nrhs);
        else if (rc == 2) hipLaunchKernelGGL((sgf::k_apply_fwd<T, 2>), g, dim3(sgf::WG), lds, st, dd, D.arena.as<T>(), sl, y, n, ts, ldt, nrhs);
        else if (rc == 3) hipLaunchKernelGGL((sgf::k_apply_fwd<T, 3>), g, dim3(sgf::WG), lds, st, dd, D.arena.as<T>(), sl, y, n, ts, ldt, nrhs);
        else hipLaunchKernelGGL((sgf::k_apply_fwd<T, 4>), g, dim3(sgf::WG), lds, st, dd, D.arena.as<T>(), sl, y, n, ts, ldt, nrhs);
      }, L.t);
      return;
    }
    launch(h, st, "mul_elim", 0, D.work.fwd_bytes + nrhs * D.work.fwd_vec, [&] {
      hipLaunchKernelGGL(sgf::k_elim_fwd<T>, dim3((unsigned)L.elim.size(), nrhs), dim3(sgf::WG), mm * sizeof(T), st,
                         D.elim.as<sgf::ElimDesc>(), D.arena.as<T>(), D.slots.as<int32_t>(), y, n, ts, ldt, mode);
    });
  };
  auto elim_bwd = [&](int li, int mode) {
    sgf::Level& L = P.levels[li];
    LevelDev& D = h->lev[li];
    int mm, mk, ms;
    maxes(L, mm, mk, ms);
    if (L.elim.empty()) return;
    if (mode == 0 && D.tiled) {
      const unsigned nf = (unsigned)D.h_tf.size();
      const size_t e = sizeof(T), mp = (D.tmax_m + 3) & ~3;
      const int rc1 = rc_for(0, std::max(D.tmax_k, 1) * e, nrhs), rc2 = rc_for(0, (mp + sgf::WG) * e, nrhs);
      launch(h, st, "apply_elim_bwd", 0, 0.5 * (cdiv(nrhs, rc1) * D.work.bwd_bytes + nrhs * D.work.bwd_vec), [&] {
        hipLaunchKernelGGL((sgf::k_tbwd_s<T, T>), dim3(cdiv(D.tmax_m, sgf::TB), nf, cdiv(nrhs, rc1)), dim3(sgf::WG),
                           (size_t)rc1 * std::max(D.tmax_k, 1) * e, st, D.tf.as<sgf::TFront>(), D.arena.as<T>(),
                           D.slots.as<int32_t>(), D.nslots.as<int32_t>(), y, n, reinterpret_cast<T*>(W.uw[li]), D.u_elems, nrhs, rc1);
      }, L.t);
      launch(h, st, "apply_elim_bwd", 0, 0.5 * (cdiv(nrhs, rc2) * D.work.bwd_bytes + nrhs * D.work.bwd_vec), [&] {
        hipLaunchKernelGGL((sgf::k_tbwd_z<T, T>), dim3(cdiv(D.tmax_m, sgf::TB), nf, cdiv(nrhs, rc2)), dim3(sgf::WG),
                           (size_t)rc2 * (mp + sgf::WG) * e, st, D.tf.as<sgf::TFront>(), D.zt.as<T>(), reinterpret_cast<T*>(W.uw[li]),
                           D.u_elems, D.slots.as<int32_t>(), y, n, nrhs, rc2);
      }, L.t);
      return;
    }
    int nb1 = 0, pw = 0;
    if (mode == 0 && band_level(h, D, false) && band1_level(h, D, nrhs, &nb1, &pw)) {
      band1_sweep<T>(h, L, D, false, nb1, pw, y, ts, st);
      return;
    }
    int k1 = 0;
    if (mode == 0 && apply1_level(h, L, D, nrhs, &k1)) {
      const int order = band_level(h, D, false) ? 1 : 0;   // the summation order of the multi-column sweeps
      launch(h, st, "apply_small_bwd", 0, D.work.bwd_bytes + D.work.bwd_vec, [&] {
        hipLaunchKernelGGL((sgf::k_apply1<T, false>), dim3((unsigned)L.elim.size()), dim3(sgf::WG),
                           (size_t)sgf::apply1_lds_elems(k1) * sizeof(T), st, D.elim.as<sgf::ElimDesc>(),
                           (const T*)D.arena.as<T>(), D.slots.as<int32_t>(), D.nslots.as<int32_t>(), y, (T*)nullptr, k1, order);
      }, L.t);
      return;
    }
    if (mode == 0 && band_level(h, D, false)) {
      const int rc = band_rc(h, D, false, nrhs);
      const int tj = band_tj(h, D);
      const size_t lds = (size_t)sgf::band_bwd_lds(D.band_m, D.band_k, D.band_bw, rc, tj) * sizeof(T);
      launch(h, st, "apply_band_bwd", 0, cdiv(nrhs, rc) * D.work.bwd_bytes + nrhs * D.work.bwd_vec, [&] {
        const dim3 g((unsigned)L.elim.size(), cdiv(nrhs, rc));
        const sgf::ElimDesc* dd = D.elim.as<sgf::ElimDesc>();
        const int32_t* sl = D.slots.as<int32_t>();
        const int32_t* ns = D.nslots.as<int32_t>();
        if (D.banded_w > 0)
          band_bwd_launch<T, true>(rc, g, lds, st, dd, D.arena.as<T>(), sl, ns, y, n, nrhs, tj, D.pk.as<T>());
        else
          band_bwd_launch<T, false>(rc, g, lds, st, dd, D.arena.as<T>(), sl, ns, y, n, nrhs, tj, (const T*)nullptr);
      }, L.t);
      return;
    }
    if (mode == 0) {
      const size_t fixed = (size_t)sgf::DB * sgf::DLD * sizeof(T);
      const int rc = rc_for(fixed, (size_t)((L.max_front_rows + 3) & ~3) * sizeof(T), nrhs);
      const size_t lds = fixed + (size_t)rc * ((L.max_front_rows + 3) & ~3) * sizeof(T);
      launch(h, st, "apply_elim_bwd", 0, cdiv(nrhs, rc) * D.work.bwd_bytes + nrhs * D.work.bwd_vec, [&] {
        const dim3 g((unsigned)L.elim.size(), cdiv(nrhs, rc));
        const sgf::ElimDesc* dd = D.elim.as<sgf::ElimDesc>();
        const int32_t* sl = D.slots.as<int32_t>();
        const int32_t* ns = D.nslots.as<int32_t>();
        if (rc == 1) hipLaunchKernelGGL((sgf::k_apply_bwd<T, 1>), g, dim3(sgf::WG), lds, st, dd, D.arena.as<T>(), sl, ns, y, n, nrhs);
        else if (rc == 2) hipLaunchKernelGGL((sgf::k_apply_bwd<T, 2>), g, dim3(sgf::WG), lds, st, dd, D.arena.as<T>(), sl, ns, y, n, nrhs);
        else if (rc == 3) hipLaunchKernelGGL((sgf::k_apply_bwd<T, 3>), g, dim3(sgf::WG), lds, st, dd, D.arena.as<T>(), sl, ns, y, n, nrhs);
        else hipLaunchKernelGGL((sgf::k_apply_bwd<T, 4>), g, dim3(sgf::WG), lds, st, dd, D.arena.as<T>(), sl, ns, y, n, nrhs);
      }, L.t);
      return;
    }
    launch(h, st, "mul_elim_t", 0, D.work.bwd_bytes + nrhs * D.work.bwd_vec, [&] {
      hipLaunchKernelGGL(sgf::k_elim_bwd<T>, dim3((unsigned)L.elim.size(), nrhs), dim3(sgf::WG),
                         (2 * mm + mk) * sizeof(T), st, D.elim.as<sgf::ElimDesc>(), D.arena.as<T>(),
                         D.slots.as<int32_t>(), D.nslots.as<int32_t>(), y, n, mode);
    });
  };
  auto sepacc = [&](int li, T sign) {
    sgf::Level& L = P.levels[li];
    LevelDev& D = h->lev[li];
    if (L.sepacc.empty()) return;
    launch(h, st, "apply_sepacc", 0, nrhs * D.work.acc_vec, [&] {
      hipLaunchKernelGGL(sgf::k_sepacc<T>, dim3((unsigned)L.sepacc.size(), nrhs), dim3(sgf::WG), 0, st,
                         D.sepacc.as<sgf::SepAcc>(), D.sepsrc.as<int64_t>(), D.slots.as<int32_t>(), ts, ldt, y, n,
                         sign);
    }, L.t);
  };
  // forward separator step (accumulation, then T_S on the compressed
  // separators) as one launch: one right-hand side, every compressed
  // separator among the accumulated ones, T_S products on the one-workgroup
  // kernel; false when these do not hold (then two launches)
  auto sepacc_comp = [&](int li) {
    sgf::Level& L = P.levels[li];
    LevelDev& D = h->lev[li];
    if (nrhs != 1 || L.sepacc.empty() || !L.acc_covers_capply || L.cap_of_acc.size() != L.sepacc.size())
      return false;
    int mm, mk, ms;
    maxes(L, mm, mk, ms);
    if (!L.capply.empty() && (ms > 256 || h->tiled_rows == 0)) return false;
    int sa = 0;
    for (const auto& a : L.sepacc) sa = std::max(sa, a.s);
    const size_t lds = 2 * (size_t)std::max(sa, sgf::WAVE) * sizeof(T);   // the small-separator path stages 64 entries
    if (lds > LDS_BYTES) return false;
    // register rows of the small-separator path sized for the level's largest separator
    const int sb = small_rows(sa);
    launch(h, st, "apply_sepacc", 0, D.work.acc_vec + D.work.capply_bytes + D.work.capply_vec, [&] {
      auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3((unsigned)L.sepacc.size()), dim3(sgf::WG), lds, st,
                           D.sepacc.as<sgf::SepAcc>(), D.sepsrc.as<int64_t>(), D.slots.as<int32_t>(), ts, y,
                           D.capacc.as<int32_t>(), D.capply.as<sgf::CompApply>(), D.tb.as<T>());
      };
      if (sb == 16) go(sgf::k_sepacc_comp<T, 16>);
      else if (sb == 32) go(sgf::k_sepacc_comp<T, 32>);
      else if (sb == 64) go(sgf::k_sepacc_comp<T, 64>);
      else go(sgf::k_sepacc_comp<T, 0>);
    }, L.t);
    return true;
  };
  auto capply = [&](int li, int mode) {
    sgf::Level& L = P.levels[li];
    LevelDev& D = h->lev[li];
    int mm, mk, ms;
    maxes(L, mm, mk, ms);
    if (L.capply.empty()) return;
    if (mode <= 1 && (ms > 256 || h->tiled_rows == 0)) {
      // large separators (or everything when every level is forced through the
      // multi-workgroup kernels): several workgroups per separator, out of place
      const unsigned nb = cdiv(ms, sgf::TB);
      const int rc = rc_for(0, ((size_t)((ms + 3) & ~3) + sgf::WG) * sizeof(T), nrhs);
      launch(h, st, "apply_comp", 0, cdiv(nrhs, rc) * D.work.capply_bytes + nrhs * D.work.capply_vec, [&] {
        hipLaunchKernelGGL(sgf::k_comp_apply_big<T>, dim3((unsigned)L.capply.size(), nb, cdiv(nrhs, rc)),
                           dim3(sgf::WG), (size_t)rc * (((ms + 3) & ~3) + sgf::WG) * sizeof(T), st,
                           D.capply.as<sgf::CompApply>(), D.tb.as<T>(), D.slots.as<int32_t>(), y, n, mode, nrhs, rc,
                           reinterpret_cast<T*>(W.cw[li]), D.c_elems);
      }, L.t);
      launch(h, st, "apply_comp", 0, 0, [&] {
        hipLaunchKernelGGL(sgf::k_comp_scatter<T>, dim3((unsigned)L.capply.size(), nrhs), dim3(sgf::WG), 0, st,
                           D.capply.as<sgf::CompApply>(), D.slots.as<int32_t>(), y, n, reinterpret_cast<T*>(W.cw[li]), D.c_elems);
      }, L.t);
      return;
    }
    if (mode <= 1) {
      const int rc = rc_for(0, 2 * (size_t)ms * sizeof(T), nrhs);
      const int sb = small_rows(ms);
      launch(h, st, "apply_comp", 0, cdiv(nrhs, rc) * D.work.capply_bytes + nrhs * D.work.capply_vec, [&] {
        auto go = [&](auto kern) {
          hipLaunchKernelGGL(kern, dim3((unsigned)L.capply.size(), cdiv(nrhs, rc)), dim3(sgf::WG),
                             2 * (size_t)rc * ms * sizeof(T), st, D.capply.as<sgf::CompApply>(), D.tb.as<T>(),
                             D.slots.as<int32_t>(), y, n, mode, nrhs, rc);
        };
        if (sb == 16) go(sgf::k_comp_apply_t<T, 16>);
        else if (sb == 32) go(sgf::k_comp_apply_t<T, 32>);
        else if (sb == 64) go(sgf::k_comp_apply_t<T, 64>);
        else go(sgf::k_comp_apply_t<T, 0>);
      }, L.t);
      return;
    }
    launch(h, st, "mul_comp", 0, 0, [&] {
      hipLaunchKernelGGL(sgf::k_comp_apply<T>, dim3((unsigned)L.capply.size(), nrhs), dim3(sgf::WG),
                         2 * ms * sizeof(T), st, D.capply.as<sgf::CompApply>(), D.cf.as<T>(), D.nbuf.as<T>(),
                         D.tau.as<T>(), D.slots.as<int32_t>(), y, n, mode);
    });
  };
  for (int li = 0; li < nl - 1; ++li) {
    if (!product) {
      elim_fwd(li, 0);
      if (!sepacc_comp(li)) {
        sepacc(li, T(-1));
        capply(li, 0);
      }
    } else {
      elim_bwd(li, 1);
      capply(li, 2);
    }
  }
  {
    sgf::Level& L = P.levels[nl - 1];
    LevelDev& D = h->lev[nl - 1];
    const int m = L.elim[0].m;
    const double tb = 2 * D.work.top_bytes * 8.0 / sizeof(T) + nrhs * D.work.top_vec;
    if (m > 0 && h->top_tiled && !product) {
      const size_t mp = (m + 3) & ~3;
      const int rc1 = rc_for(0, m * sizeof(double), nrhs), rc2 = rc_for(0, (mp + sgf::WG) * sizeof(double), nrhs);
      launch(h, st, "apply_top", 0, 0.5 * tb, [&] {
        hipLaunchKernelGGL((sgf::k_tfwd_z<T, double>), dim3(cdiv(m, sgf::TB), 1, cdiv(nrhs, rc1)), dim3(sgf::WG),
                           (size_t)rc1 * m * sizeof(double), st, h->d_toptf.as<sgf::TFront>(), h->topz.as<double>(),
                           D.slots.as<int32_t>(), y, n, reinterpret_cast<double*>(W.topu), (int64_t)m, nrhs, rc1);
      }, L.t);
      launch(h, st, "apply_top", 0, 0.5 * tb, [&] {
        hipLaunchKernelGGL((sgf::k_tbwd_z<T, double>), dim3(cdiv(m, sgf::TB), 1, cdiv(nrhs, rc2)), dim3(sgf::WG),
                           (size_t)rc2 * (mp + sgf::WG) * sizeof(double), st, h->d_toptf.as<sgf::TFront>(),
                           h->topz.as<double>(), reinterpret_cast<double*>(W.topu), (int64_t)m, D.slots.as<int32_t>(), y, n, nrhs,
                           rc2);
      }, L.t);
    } else if (m > 0) {
      if ((size_t)2 * m * sizeof(double) > LDS_BYTES)
        throw SgfError(SGF_EINVAL, "top node too large for the one-workgroup top kernel");
      const size_t staged_lds = ((size_t)2 * m + (size_t)m * (m + 1)) * sizeof(double);
      const int staged = !product && staged_lds <= LDS_BYTES;
      launch(h, st, "apply_top", 0, tb, [&] {
        hipLaunchKernelGGL((sgf::k_top<T, double>), dim3(1, nrhs), dim3(sgf::WG),
                           staged ? staged_lds : 2 * m * sizeof(double), st, h->d_topdesc.as<sgf::ElimDesc>(),
                           h->top64.as<double>(), D.slots.as<int32_t>(), y, n, product ? 1 : 0, staged);
      }, L.t);
    }
  }
  for (int li = nl - 2; li >= 0; --li) {
    if (!product) {
      capply(li, 1);
      elim_bwd(li, 0);
    } else {
      capply(li, 3);
      elim_fwd(li, 1);
      sepacc(li, T(1));
    }
  }
}

// Records body(stream) on the handle's private stream as a graph and
// instantiates it.  No event records inside (profiling paused); the body
// must launch kernels only (no memset nodes).
template <typename F>
hipGraphExec_t capture_graph(sgf_handle h, F&& body) {
  if (!h->cap_stream) HIP_CHECK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
  const bool prof = h->prof.on;
  h->prof.on = false;
  h->capturing = true;
  HIP_CHECK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
  hipGraph_t graph = nullptr;
  try {
    body(h->cap_stream);
  } catch (...) {
    (void)hipStreamEndCapture(h->cap_stream, &graph);
    if (graph) (void)hipGraphDestroy(graph);
    h->prof.on = prof;
    h->capturing = false;
    throw;
  }
  h->prof.on = prof;
  h->capturing = false;
  HIP_CHECK(hipStreamEndCapture(h->cap_stream, &graph));
  hipGraphExec_t exec = nullptr;
  const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  HIP_CHECK(e);
  return exec;
}

// ext: work vectors supplied by the caller (the allocation-free apply): no
// buffer is grown, no graph is captured, every kernel is launched directly.
template <typename T>
void apply_impl(sgf_handle h, int nrhs, const double* r, int64_t ldr, double* z, int64_t ldz, bool product,
                hipStream_t st, const ApplyWork* ext = nullptr) {
  const int64_t n = h->plan.n;
  if (!ext) ensure_work<T>(h, nrhs);
  const ApplyWork W = ext ? *ext : handle_work(h);
  T* yw = reinterpret_cast<T*>(W.y);
  dim3 g(cdiv(n, sgf::WG), nrhs);
  const double vb = (double)n * nrhs * (8.0 + sizeof(T)) + 8.0 * n;
  auto body = [&](hipStream_t s) {
    launch(h, s, "apply_perm", 0, vb, [&] {
      hipLaunchKernelGGL((sgf::k_gather_perm<double, T>), g, dim3(sgf::WG), 0, s, h->d_perm.as<int64_t>(), n, r, ldr,
                         yw, n);
    });
    run_sweeps<T>(h, nrhs, product, s, W);
    launch(h, s, "apply_perm", 0, vb, [&] {
      hipLaunchKernelGGL((sgf::k_scatter_perm<T, double>), g, dim3(sgf::WG), 0, s, h->d_perm.as<int64_t>(), n,
                         yw, n, z, ldz);
    });
  };
  if (!h->use_graph || h->capturing || ext) {
    body(st);
    HIP_CHECK(hipGetLastError());
    return;
  }
  auto& G = h->ag;
  if (!(G.exec && G.nrhs == nrhs && G.r == r && G.ldr == ldr && G.z == z && G.ldz == ldz && G.product == product &&
        G.epoch == h->epoch)) {
    if (G.exec) (void)hipGraphExecDestroy(G.exec);
    G.exec = nullptr;
    hipGraphExec_t exec = capture_graph(h, body);
    G.exec = exec;
    G.nrhs = nrhs;
    G.r = r;
    G.ldr = ldr;
    G.z = z;
    G.ldz = ldz;
    G.product = product;
    G.epoch = h->epoch;
  }
  launch(h, st, "apply_graph", 0, h->apply_bytes * nrhs, [&] { HIP_CHECK(hipGraphLaunch(G.exec, st)); });
}

void apply_any(sgf_handle h, int nrhs, const double* r, int64_t ldr, double* z, int64_t ldz, bool product,
               hipStream_t st) {
  if (h->esz == 8) apply_impl<double>(h, nrhs, r, ldr, z, ldz, product, st);
  else apply_impl<float>(h, nrhs, r, ldr, z, ldz, product, st);
}

void dot_cols(sgf_handle h, const double* a, const double* b, int nrhs, double* out, hipStream_t st) {
  const int64_t n = h->plan.n;
  const int nb = (int)std::min<int64_t>(1024, cdiv(n, sgf::WG));
  launch(h, st, "cg_dot", 0, 16.0 * n * nrhs, [&] {
    hipLaunchKernelGGL(sgf::k_dot_partial, dim3(nb, nrhs), dim3(sgf::WG), 0, st, a, n, b, n, n,
                       h->cg_part.as<double>());
  });
  launch(h, st, "cg_reduce", 0, 8.0 * nb * nrhs, [&] {
    hipLaunchKernelGGL(sgf::k_reduce, dim3(nrhs), dim3(sgf::WG), 0, st, h->cg_part.as<double>(), nb, out, 1);
  });
}

// Device memory held by the handle.
int64_t device_bytes(sgf_handle h) {
  int64_t b = 0;
  for (const DevBuf* x : {&h->d_perm, &h->d_rowptr, &h->d_colidx, &h->d_vals, &h->d_csrdst, &h->d_coords,
                          &h->d_basis, &h->d_fail,
                          &h->d_ctr, &h->d_zero_idx,
                          &h->y, &h->tscr, &h->cg_r, &h->cg_z, &h->cg_p, &h->cg_ap, &h->cg_x, &h->cg_part, &h->cg_st,
                          &h->cg_scal, &h->top64, &h->topz, &h->topu, &h->d_topdesc, &h->d_toptf})
    b += x->bytes;
  for (const auto& D : h->lev)
    for (const DevBuf* x : {&D.arena, &D.scratch, &D.cf, &D.nbuf, &D.ltphi, &D.tau, &D.phi, &D.rank, &D.elim,
                            &D.pairs, &D.schur, &D.comp, &D.compnbr, &D.sepacc, &D.sepsrc, &D.capply, &D.slots,
                            &D.nslots, &D.blkmap, &D.phimap, &D.slotptr, &D.phioff, &D.tb, &D.active, &D.tofcomp,
                            &D.tf, &D.zt, &D.uw, &D.ctf, &D.elim_order, &D.comp_order, &D.cw, &D.band_list, &D.pk,
                            &D.fixrank})
      b += x->bytes;
  return b;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

void sgf_default_options(sgf_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->dim = 2;
  o->grid[0] = o->grid[1] = o->grid[2] = 1;
  o->dofs_per_node = 1;
  o->q = 1;
  o->leaf = 8;
  o->scheme = SGF_NEST_ALL_ALL;
  o->compress = 1;
  o->compress_from_level = 1;
  o->stop_rule = SGF_STOP_ROOT;
  o->precision = SGF_FP64;
  o->tiled_min_rows = -1;
  o->rank_tol = 0.0;
}

const char* sgf_status_str(sgf_status s) {
  switch (s) {
    case SGF_OK: return "ok";
    case SGF_EINVAL: return "invalid argument";
    case SGF_ENOTSPD: return "matrix not positive definite";
    case SGF_ENOMEM: return "out of memory";
    case SGF_EDEVICE: return "device error";
    case SGF_ENOCONV: return "no convergence";
    case SGF_ESTATE: return "call out of order";
  }
  return "unknown status";
}

const char* sgf_last_error(void) { return g_last_error.c_str(); }

sgf_status sgf_analyze(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, const double* coords,
                       const sgf_options* opt, sgf_handle* out) {
  if (!out) return fail(SGF_EINVAL, "out is NULL");
  *out = nullptr;
  std::unique_ptr<sgf_handle_s> h(new (std::nothrow) sgf_handle_s());
  if (!h) return fail(SGF_ENOMEM, "handle allocation failed");
  sgf_status st = guard([&] {
    check_options(opt, n);
    if (!row_ptr || !col_idx) throw SgfError(SGF_EINVAL, "NULL input array");
    if (!coords && opt->q != 0)
      throw SgfError(SGF_EINVAL, "coordinates are needed for polynomial degree q > 0 (q = 0 or a user basis needs none)");
    sgf::Options& o = h->plan.opt;
    o.dim = opt->dim;
    for (int a = 0; a < 3; ++a) o.grid[a] = a < opt->dim ? opt->grid[a] : 1;
    o.dpn = opt->dofs_per_node;
    o.q = opt->q;
    o.leaf = opt->leaf;
    o.scheme = opt->scheme;
    o.compress = opt->compress;
    o.compress_from_level = std::max(1, opt->compress_from_level);
    o.stop_rule = opt->stop_rule;
    o.precision = opt->precision;
    o.rank_tol = opt->rank_tol > 0 ? opt->rank_tol
                                   : (opt->precision == SGF_FP64 ? 1e-12 : opt->precision == SGF_FP32 ? 1e-6 : 1e-2);
    h->tiled_rows = opt->tiled_min_rows < 0 ? 1024 : opt->tiled_min_rows;
    h->esz = opt->precision == SGF_FP64 ? 8 : 4;
    h->plan.n = n;
    h->plan.n_nodes = n / o.dpn;
    h->plan.pi = sgf::poly_cols(o.dim, o.q, o.dpn);
    if (row_ptr[0] != 0) throw SgfError(SGF_EINVAL, "row_ptr[0] must be 0");
    for (int64_t i = 0; i < n; ++i)
      if (row_ptr[i + 1] < row_ptr[i]) throw SgfError(SGF_EINVAL, "row_ptr not monotone");
    h->nnz = row_ptr[n];
    h->h_rowptr.assign(row_ptr, row_ptr + n + 1);
    h->h_colidx.assign(col_idx, col_idx + h->nnz);
    if (coords) h->h_coords.assign(coords, coords + h->plan.n_nodes * o.dim);
    for (int a = 0; a < 3; ++a) {
      h->plan.cmin[a] = 0;
      h->plan.cmax[a] = 0;
    }
    for (int a = 0; coords && a < o.dim; ++a) {
      double lo = coords[a], hi = coords[a];
      for (int64_t v = 0; v < h->plan.n_nodes; ++v) {
        lo = std::min(lo, coords[v * o.dim + a]);
        hi = std::max(hi, coords[v * o.dim + a]);
      }
      h->plan.cmin[a] = lo;
      h->plan.cmax[a] = hi;
    }
    sgf::plan_level1(h->plan, row_ptr, col_idx);
  });
  if (st != SGF_OK) return st;
  *out = h.release();
  return SGF_OK;
}

sgf_status sgf_factorize_numeric(sgf_handle h, const double* vals, void* stream) {
  if (!h || !vals) return fail(SGF_EINVAL, "NULL handle or values");
  hipStream_t st = (hipStream_t)stream;
  return guard([&] {
    if (h->esz == 8) factor_numeric<double>(h, vals, st);
    else factor_numeric<float>(h, vals, st);
  });
}

sgf_status sgf_autotune(sgf_handle h, const double* vals, int32_t napply, int32_t* modes_out, void* stream) {
  if (!h || !vals || napply < 0) return fail(SGF_EINVAL, "bad autotune arguments");
  hipStream_t st = (hipStream_t)stream;
  return guard([&] {
    const int64_t n = h->plan.n;
    DevBuf r, z;
    r.ensure(n * sizeof(double));
    z.ensure(n * sizeof(double));
    HIP_CHECK(hipMemsetAsync(r.p, 0, n * sizeof(double), st));
    const bool prof_was = h->prof.on;
    h->prof.drain();
    const auto saved = h->prof.stats;
    struct Restore {
      sgf_handle h;
      bool on;
      std::vector<sgf_kernel_stat> stats;
      bool graph;
      ~Restore() {
        h->force_mode = -1;
        h->use_graph = graph;
        h->prof.on = on;
        h->prof.stats = stats;
        for (auto& D : h->lev) D.uploaded = false;
      }
    } restore{h, prof_was, saved, h->use_graph};
    h->use_graph = false;   // per-level apply timings need direct launches
    // every candidate runs three times, interleaved, and keeps its fastest
    // time per level (a single trial is noisy, the first pays cold memory)
    const int candidates[] = {0, 1, 8, 16, 32};
    const int nc = 5, reps = 3;
    std::vector<std::vector<double>> cost(nc);   // [candidate][level]
    std::vector<std::vector<char>> honored(nc);  // the level really ran that candidate
    for (int trial = 0; trial < nc * reps; ++trial) {
      const int ci = trial % nc, c = candidates[ci];
      h->force_mode = c;
      h->level_mode.clear();
      for (auto& D : h->lev) D.uploaded = false;
      h->prof.stats.clear();
      h->prof.on = true;
      if (h->esz == 8) factor_numeric<double>(h, vals, st);
      else factor_numeric<float>(h, vals, st);
      apply_any(h, 1, r.as<double>(), n, z.as<double>(), n, false, st);
      h->prof.drain();
      const int nl = (int)h->plan.levels.size();
      std::vector<double> lc(nl, 0.0);
      std::vector<char> ok(nl, 0);
      for (int li = 0; li < nl; ++li) {
        const auto& L = h->plan.levels[li];
        if (L.top || L.elim.empty()) continue;
        ok[li] = (c == 0) == h->lev[li].tiled && (c == 1) == (h->lev[li].banded_w > 0);
        char tag[48];
        for (const auto& k : h->prof.stats) {
          const std::string nm(k.name);
          std::snprintf(tag, sizeof(tag), "@L%d", L.t);
          const size_t at = nm.find('@');
          if (at == std::string::npos || nm.substr(at) != tag) continue;
          const std::string base = nm.substr(0, at);
          if (base == "elim" || base.rfind("elim_", 0) == 0) lc[li] += k.ms;
          else if (base == "apply_elim_fwd" || base == "apply_elim_bwd" || base == "apply_band_fwd" ||
                   base == "apply_band_bwd")
            lc[li] += napply * k.ms;
        }
      }
      if (cost[ci].empty()) {
        cost[ci] = lc;
        honored[ci] = ok;
      } else {
        for (int li = 0; li < nl; ++li) cost[ci][li] = std::min(cost[ci][li], lc[li]);
      }
    }
    const int nl = (int)h->plan.levels.size();
    std::vector<int32_t> modes(nl, -1);
    for (int li = 0; li < nl; ++li) {
      double best = 0;
      for (size_t c = 0; c < cost.size(); ++c) {
        if (li >= (int)cost[c].size() || !honored[c][li]) continue;
        if (modes[li] == -1 || cost[c][li] < best) {
          best = cost[c][li];
          modes[li] = candidates[c];
        }
      }
    }
    h->level_mode = modes;
    h->factored = false;
    if (modes_out)
      for (int li = 0; li < nl; ++li) modes_out[li] = modes[li];
  });
}

sgf_status sgf_factorize(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, const double* vals,
                         const double* coords, const sgf_options* opt, void* stream, sgf_handle* out) {
  sgf_handle h = nullptr;
  sgf_status s = sgf_analyze(n, row_ptr, col_idx, coords, opt, &h);
  if (s != SGF_OK) return s;
  s = sgf_factorize_numeric(h, vals, stream);
  if (s != SGF_OK) {
    sgf_destroy(h);
    if (out) *out = nullptr;
    return s;
  }
  *out = h;
  return SGF_OK;
}

sgf_status sgf_apply(sgf_handle h, int32_t nrhs, const double* r, int64_t ldr, double* z, int64_t ldz, void* stream) {
  if (!h || !r || !z || nrhs < 1) return fail(SGF_EINVAL, "bad apply arguments");
  if (!h->factored) return fail(SGF_ESTATE, "apply before a successful factorization");
  if (ldr < h->plan.n || ldz < h->plan.n) return fail(SGF_EINVAL, "leading dimension below n");
  return guard([&] { apply_any(h, nrhs, r, ldr, z, ldz, false, (hipStream_t)stream); });
}

}  // extern "C"

// Device scratch of the allocation-free apply: one array per GPU, held from
// the library's load until the process ends.  Host code never passes this
// name to a kernel (on the host it only stands for the symbol): the device
// address of each GPU's copy is looked up once per device and kept.
static __device__ __align__(256) unsigned char scratch[SGF_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

void* scratch_ptr() {
  int dev = 0;
  HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) throw SgfError(SGF_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw SgfError(SGF_EDEVICE, "no device address for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

// The apply's work vectors carved out of `base` (256-byte aligned pieces,
// the sizes ensure_work would allocate); bytes needed in *need.
ApplyWork carve_work(sgf_handle h, int nrhs, unsigned char* base, size_t* need) {
  ApplyWork w;
  const size_t e = h->esz;
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    void* p = base + off;
    off += (bytes + 255) & ~(size_t)255;
    return p;
  };
  w.y = take((size_t)h->plan.n * nrhs * e);
  w.tscr = take((size_t)std::max<int64_t>(h->max_t, 1) * nrhs * e);
  if ((int)h->lev.size() > ApplyWork::MAXL) throw SgfError(SGF_EINVAL, "too many levels for the allocation-free apply");
  for (size_t li = 0; li < h->lev.size(); ++li) {
    const LevelDev& D = h->lev[li];
    if (D.tiled && D.uploaded) w.uw[li] = take((size_t)std::max<int64_t>(D.u_elems, 1) * nrhs * e);
    if (D.uploaded) w.cw[li] = take((size_t)std::max<int64_t>(D.c_elems, 1) * nrhs * e);
  }
  if (h->top_tiled) w.topu = take((size_t)h->top_R * nrhs * sizeof(double));
  *need = off;
  return w;
}
}  // namespace

extern "C" {

sgf_status sgf_apply_noalloc(sgf_handle h, int32_t nrhs, const double* r, int64_t ldr, double* z, int64_t ldz,
                             void* stream) {
  if (!h || !r || !z || nrhs < 1) return fail(SGF_EINVAL, "bad apply arguments");
  if (!h->factored) return fail(SGF_ESTATE, "apply before a successful factorization");
  if (ldr < h->plan.n || ldz < h->plan.n) return fail(SGF_EINVAL, "leading dimension below n");
  return guard([&] {
    size_t need = 0;
    (void)carve_work(h, nrhs, nullptr, &need);   // sizes only
    if (need > SGF_NOALLOC_SCRATCH_BYTES)
      throw SgfError(SGF_EINVAL, "allocation-free apply needs " + std::to_string(need) + " bytes of scratch for " +
                                     std::to_string(nrhs) + " columns; the static scratch holds " +
                                     std::to_string((size_t)SGF_NOALLOC_SCRATCH_BYTES));
    unsigned char* base = static_cast<unsigned char*>(scratch_ptr());
    const ApplyWork w = carve_work(h, nrhs, base, &need);
    const bool prof = h->prof.on;
    h->prof.on = false;   // no events: launches only
    try {
      if (h->esz == 8) apply_impl<double>(h, nrhs, r, ldr, z, ldz, false, (hipStream_t)stream, &w);
      else apply_impl<float>(h, nrhs, r, ldr, z, ldz, false, (hipStream_t)stream, &w);
    } catch (...) {
      h->prof.on = prof;
      throw;
    }
    h->prof.on = prof;
  });
}

sgf_status sgf_multiply(sgf_handle h, int32_t nrhs, const double* v, int64_t ldv, double* y, int64_t ldy,
                        void* stream) {
  if (!h || !v || !y || nrhs < 1) return fail(SGF_EINVAL, "bad multiply arguments");
  if (!h->factored) return fail(SGF_ESTATE, "multiply before a successful factorization");
  if (ldv < h->plan.n || ldy < h->plan.n) return fail(SGF_EINVAL, "leading dimension below n");
  return guard([&] { apply_any(h, nrhs, v, ldv, y, ldy, true, (hipStream_t)stream); });
}

sgf_status sgf_spmv(sgf_handle h, const double* v, double* y, void* stream) {
  if (!h || !v || !y) return fail(SGF_EINVAL, "bad spmv arguments");
  if (!h->dev_static) return fail(SGF_ESTATE, "spmv before factorization");
  return guard([&] {
    const int64_t n = h->plan.n;
    spmv_launch(h, v, n, y, n, 1, nullptr, (hipStream_t)stream);
    HIP_CHECK(hipGetLastError());
  });
}

sgf_status sgf_pcg_solve(sgf_handle h, int32_t nrhs, const double* b, int64_t ldb, double* x, int64_t ldx,
                         double rtol, int32_t maxit, int32_t* iters, double* relres, void* stream) {
  if (!h || !b || !x || nrhs < 1 || nrhs > 256 || maxit < 0 || !iters || !relres)
    return fail(SGF_EINVAL, "bad pcg arguments");
  if (!h->factored) return fail(SGF_ESTATE, "pcg before a successful factorization");
  if (ldb < h->plan.n || ldx < h->plan.n) return fail(SGF_EINVAL, "leading dimension below n");
  hipStream_t st = (hipStream_t)stream;
  bool all_conv = true;
  sgf_status s = guard([&] {
    const int64_t n = h->plan.n;
    const size_t vb = (size_t)n * nrhs * sizeof(double);
    h->cg_r.ensure(vb);
    h->cg_z.ensure(vb);
    h->cg_p.ensure(vb);
    h->cg_ap.ensure(vb);
    h->cg_x.ensure(vb);
    const int nbs = (int)std::min<int64_t>(1024, cdiv(n, sgf::WG));
    const int nbspmv = (int)spmv_blocks(h);
    h->cg_part.ensure((size_t)std::max(nbs, nbspmv) * nrhs * sizeof(double));
    h->cg_st.ensure(8 * nrhs * sizeof(double));
    h->cg_scal.ensure(2 * nrhs * sizeof(double));
    double* r = h->cg_r.as<double>();
    double* z = h->cg_z.as<double>();
    double* p = h->cg_p.as<double>();
    double* Ap = h->cg_ap.as<double>();
    double* xi = h->cg_x.as<double>();   // iterate, copied to x at the end
    double* stv = h->cg_st.as<double>();
    double* sc = h->cg_scal.as<double>();
    for (int c = 0; c < nrhs; ++c)
      HIP_CHECK(hipMemcpyAsync(r + c * n, b + c * ldb, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    HIP_CHECK(hipMemsetAsync(xi, 0, vb, st));
    HIP_CHECK(hipMemsetAsync(p, 0, vb, st));
    auto copy_out = [&] {
      HIP_CHECK(hipMemcpy2DAsync(x, ldx * sizeof(double), xi, n * sizeof(double), n * sizeof(double), nrhs,
                                 hipMemcpyDeviceToDevice, st));
    };
    std::vector<double> hst(8 * nrhs, 0.0), bn(nrhs), rr(nrhs), act(nrhs);
    dot_cols(h, r, r, nrhs, sc, st);
    HIP_CHECK(hipMemcpyAsync(bn.data(), sc, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    std::vector<int> active(nrhs);
    int nactive = 0;
    for (int c = 0; c < nrhs; ++c) {
      bn[c] = std::sqrt(bn[c]);
      active[c] = bn[c] > 0;
      nactive += active[c];
      iters[c] = 0;
      relres[c] = 0.0;
      hst[8 * c + 0] = std::numeric_limits<double>::infinity();   // first beta = 0
      hst[8 * c + 5] = active[c];
    }
    HIP_CHECK(hipMemcpyAsync(stv, hst.data(), 8 * nrhs * sizeof(double), hipMemcpyHostToDevice, st));
    if (nactive == 0) {
      copy_out();
      HIP_CHECK(hipStreamSynchronize(st));
      return;
    }
    dim3 gv(cdiv(n, sgf::WG), nrhs);
    const double spmv_bytes = cdiv(nrhs, 8) * (12.0 * h->nnz + 8.0 * (n + 1)) + nrhs * 24.0 * n;
    // one iteration: z = M r, rz, beta, p = z + beta p, Ap and p.Ap, alpha,
    // x += alpha p, r -= alpha Ap, rr -> sc (the only value the host reads)
    auto iteration = [&](hipStream_t s) {
      apply_any(h, nrhs, r, n, z, n, false, s);
      dot_cols(h, r, z, nrhs, sc, s);
      launch(h, s, "cg_axpy", 0, 24.0 * n * nrhs, [&] {
        hipLaunchKernelGGL(sgf::k_cg_update_p, gv, dim3(sgf::WG), 0, s, p, z, n, n, stv, sc);
      });
      launch(h, s, "cg_spmv", 0, spmv_bytes, [&] { spmv_launch(h, p, n, Ap, n, nrhs, h->cg_part.as<double>(), s); });
      launch(h, s, "cg_reduce", 0, 8.0 * nbspmv * nrhs, [&] {
        hipLaunchKernelGGL(sgf::k_reduce, dim3(nrhs), dim3(sgf::WG), 0, s, h->cg_part.as<double>(), nbspmv, stv + 1, 8);
      });
      launch(h, s, "cg_axpy", 0, 48.0 * n * nrhs, [&] {
        hipLaunchKernelGGL(sgf::k_cg_update_xr, gv, dim3(sgf::WG), 0, s, xi, n, r, n, p, Ap, n, n, stv, sc);
      });
      dot_cols(h, r, r, nrhs, sc, s);
    };
    const double iter_bytes = h->apply_bytes * nrhs + spmv_bytes + 2 * 16.0 * n * nrhs + 72.0 * n * nrhs;
    const void* bufs[8] = {r, z, p, Ap, stv, sc, h->cg_part.p, xi};
    hipGraphExec_t exec = nullptr;
    if (h->use_graph) {
      ensure_work_any(h, nrhs);   // allocations before a capture, not inside it
      // drop graphs recorded on older buffers or factors; reuse or record one
      // for this rhs count (at most four kept, least recently used evicted)
      auto& IG = h->ig;
      for (size_t i = 0; i < IG.size();) {
        if (IG[i].epoch != h->epoch || !std::equal(bufs, bufs + 8, IG[i].bufs)) {
          (void)hipGraphExecDestroy(IG[i].exec);
          IG.erase(IG.begin() + i);
        } else {
          ++i;
        }
      }
      for (auto& g : IG)
        if (g.nrhs == nrhs) exec = g.exec, g.used = ++h->ig_clock;
      if (!exec) {
        if (IG.size() >= 4) {
          auto old = std::min_element(IG.begin(), IG.end(), [](const auto& a, const auto& b) { return a.used < b.used; });
          (void)hipGraphExecDestroy(old->exec);
          IG.erase(old);
        }
        sgf_handle_s::IterGraph g;
        g.exec = capture_graph(h, iteration);
        g.nrhs = nrhs;
        g.epoch = h->epoch;
        g.used = ++h->ig_clock;
        std::copy(bufs, bufs + 8, g.bufs);
        IG.push_back(g);
        exec = g.exec;
      }
    }
    for (int it = 1; it <= maxit; ++it) {
      if (exec) {
        launch(h, st, "pcg_iteration_graph", 0, iter_bytes, [&] { HIP_CHECK(hipGraphLaunch(exec, st)); });
      } else {
        iteration(st);
      }
      HIP_CHECK(hipMemcpyAsync(rr.data(), sc, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
      HIP_CHECK(hipStreamSynchronize(st));
      bool changed = false;
      nactive = 0;
      for (int c = 0; c < nrhs; ++c) {
        if (!active[c]) continue;
        double rel = std::sqrt(std::max(rr[c], 0.0)) / bn[c];
        iters[c] = it;
        relres[c] = rel;
        if (rel < rtol) {
          active[c] = 0;
          changed = true;
        } else {
          ++nactive;
        }
      }
      if (changed) {
        for (int c = 0; c < nrhs; ++c) {
          act[c] = active[c];
          HIP_CHECK(hipMemcpyAsync(stv + 8 * c + 5, &act[c], sizeof(double), hipMemcpyHostToDevice, st));
        }
        HIP_CHECK(hipStreamSynchronize(st));
      }
      if (nactive == 0) break;
      HIP_CHECK(hipGetLastError());
    }
    copy_out();
    HIP_CHECK(hipStreamSynchronize(st));
    for (int c = 0; c < nrhs; ++c)
      if (active[c]) all_conv = false;
  });
  if (s != SGF_OK) return s;
  if (!all_conv) return fail(SGF_ENOCONV, "CG reached maxit before the tolerance");
  return SGF_OK;
}

sgf_status sgf_release(sgf_handle h) {
  if (!h) return fail(SGF_EINVAL, "NULL handle");
  return guard([&] {
    h->drop_graph();
    h->lev.clear();
    for (DevBuf* b : {&h->d_perm, &h->d_rowptr, &h->d_colidx, &h->d_vals, &h->d_csrdst, &h->d_coords, &h->d_basis,
                      &h->d_fail,
                      &h->d_ctr, &h->d_zero_idx,
                      &h->y, &h->tscr, &h->cg_r, &h->cg_z, &h->cg_p, &h->cg_ap, &h->cg_x, &h->cg_part, &h->cg_st,
                      &h->cg_scal, &h->top64, &h->topz, &h->topu, &h->d_topdesc, &h->d_toptf})
      b->release();
    h->plan.levels.resize(1);
    h->plan.parts.resize(1);
    h->dev_static = false;
    h->factored = false;
    h->top_tiled = false;
    ++h->epoch;
  });
}

sgf_status sgf_estimate_bytes(sgf_handle h, int32_t nrhs, int64_t* bytes) {
  if (!h || !bytes || nrhs < 1) return fail(SGF_EINVAL, "bad estimate arguments");
  return guard([&] {
    const double e = (double)h->esz;
    const int64_t n = h->plan.n;
    double work = (double)nrhs * (n * e + 5.0 * n * 8 + 3.0 * n * 8);
    if (h->factored) {
      *bytes = device_bytes(h) + (int64_t)work;
      return;
    }
    // plan every level with the largest rank each separator can have
    // (min(|B|, columns of N)): an upper bound of the factor's memory
    sgf::Plan& P = h->plan;
    P.levels.resize(1);
    P.parts.resize(1);
    for (size_t q = 1; q < h->lev.size(); ++q) h->lev[q].uploaded = false;
    P.max_node = 0;
    for (int sz : P.levels[0].size) P.max_node = std::max<int64_t>(P.max_node, sz);
    std::vector<sgf::CopyDesc> bm, pm;
    double tot = (double)h->nnz * (8 + 8 + 4) + (n + 1) * 8.0 + n * 8.0 + (double)P.n_nodes * P.opt.dim * 8;
    double tmax = 0;
    for (;;) {
      sgf::Level& L = P.levels.back();
      tot += e * (double)(L.front_elems + L.blk_elems + L.scratch_elems + L.cf_elems + L.n_elems + L.ltphi_elems +
                          L.tau_elems + L.phi_elems);
      tmax = std::max<double>(tmax, (double)L.t_elems);
      if (L.top) {
        const double R = L.elim.empty() ? 0 : L.elim[0].m;
        tot += 2.0 * R * R * 8 + (double)nrhs * R * 8;
        break;
      }
      if (level_tiled(h, L))
        for (const auto& d : L.elim) tot += e * ((double)d.m * d.m + (double)d.m * nrhs);
      {
        // packed copies of a level eliminated by the banded kernel
        bool banded = !L.elim.empty();
        double pk = 0;
        for (const auto& d : L.elim) {
          const int b = std::min(d.bw, std::max(d.m - 1, 0));
          if (b >= 32 || d.k > sgf::BE_KMAX) banded = false;
          pk += (double)sgf::band_pk_elems(d.m, d.k, b);
        }
        if (banded) tot += e * pk;
      }
      L.rank.assign(L.comp.size(), 0);
      for (size_t c = 0; c < L.comp.size(); ++c) {
        L.rank[c] = std::min(L.comp[c].s, L.comp[c].c);
        tot += e * (double)L.comp[c].s * L.comp[c].s;   // T_B if it compresses
      }
      sgf::plan_next_level(P, bm, pm);
    }
    P.levels.resize(1);
    P.parts.resize(1);
    // descriptor tables and index maps: a few percent of the factor
    *bytes = (int64_t)(1.05 * tot + work + tmax * nrhs * e);
  });
}

sgf_status sgf_get_info(sgf_handle h, sgf_info* info) {
  if (!h || !info) return fail(SGF_EINVAL, "NULL handle or info");
  std::memset(info, 0, sizeof(*info));
  info->levels = (int32_t)h->plan.levels.size();
  info->n = h->plan.n;
  if (h->factored) info->top_size = h->plan.levels.back().elim[0].m;
  info->factor_entries = h->factor_entries;
  info->factor_bytes = h->factor_bytes;
  info->compressed = h->compressed;
  info->factor_flops = h->factor_flops;
  info->apply_bytes = h->apply_bytes;
  info->failed_cluster = h->failed_cluster;
  info->failed_level = h->failed_level;
  info->device_bytes = device_bytes(h);
  return SGF_OK;
}

sgf_status sgf_get_perm(sgf_handle h, int64_t* perm) {
  if (!h || !perm) return fail(SGF_EINVAL, "NULL argument");
  std::memcpy(perm, h->plan.perm.data(), h->plan.n * sizeof(int64_t));
  return SGF_OK;
}

sgf_status sgf_get_level(sgf_handle h, int32_t level, int32_t* count, int32_t* cell_ids, int32_t* types,
                         int32_t* sizes, int32_t* ranks) {
  if (!h || !count) return fail(SGF_EINVAL, "NULL argument");
  if (level < 1 || level > (int)h->plan.levels.size()) return fail(SGF_EINVAL, "level out of range");
  const sgf::Level& L = h->plan.levels[level - 1];
  const int nc = (int)L.cell.size();
  *count = nc;
  for (int c = 0; c < nc; ++c) {
    if (cell_ids) cell_ids[c] = (int32_t)L.cell[c];
    if (types) types[c] = L.top ? 0 : L.type[c];
    if (sizes) sizes[c] = L.size[c];
    if (ranks) {
      bool elim = L.top || L.type[c] == 0;
      ranks[c] = elim ? 0 : (L.rank.empty() ? L.size[c] : L.post_size(c));
    }
  }
  return SGF_OK;
}

}  // extern "C"

namespace {
template <typename T>
std::vector<double> read_block(const DevBuf& b, int64_t off, int64_t elems) {
  std::vector<T> tmp((size_t)std::max<int64_t>(elems, 0));
  if (elems > 0) {
    if ((size_t)(off + elems) * sizeof(T) > b.bytes) throw SgfError(SGF_EINVAL, "factor block outside its buffer");
    HIP_CHECK(hipMemcpy(tmp.data(), b.as<T>() + off, elems * sizeof(T), hipMemcpyDeviceToHost));
  }
  return std::vector<double>(tmp.begin(), tmp.end());
}
std::vector<double> read_any(sgf_handle h, const DevBuf& b, int64_t off, int64_t elems) {
  return h->esz == 8 ? read_block<double>(b, off, elems) : read_block<float>(b, off, elems);
}
}  // namespace

extern "C" {

sgf_status sgf_block_count(sgf_handle h, int32_t level, int32_t* n_elim, int32_t* n_comp) {
  if (!h || !n_elim || !n_comp) return fail(SGF_EINVAL, "NULL argument");
  if (!h->factored) return fail(SGF_ESTATE, "the handle is not factored");
  if (level < 1 || level > (int)h->plan.levels.size()) return fail(SGF_EINVAL, "level out of range");
  const sgf::Level& L = h->plan.levels[level - 1];
  *n_elim = L.top ? 1 : (int32_t)L.elim.size();
  *n_comp = L.top ? 0 : (int32_t)L.capply.size();
  return SGF_OK;
}

sgf_status sgf_export_block(sgf_handle h, int32_t level, int32_t index, sgf_block* info, double* L_out,
                            double* W_out, double* V_out, double* tau_out, double* rdiag_out) {
  if (!h || !info) return fail(SGF_EINVAL, "NULL argument");
  if (!h->factored) return fail(SGF_ESTATE, "the handle is not factored");
  if (level < 1 || level > (int)h->plan.levels.size()) return fail(SGF_EINVAL, "level out of range");
  return guard([&] {
    const sgf::Level& L = h->plan.levels[level - 1];
    const LevelDev& D = h->lev[level - 1];
    *info = sgf_block{};
    HIP_CHECK(hipDeviceSynchronize());
    if (L.top) {
      if (index != 0) throw SgfError(SGF_EINVAL, "the top level has one block");
      const int R = L.elim[0].m;
      info->kind = SGF_BLOCK_TOP;
      info->cell = -1;
      info->m = R;
      if (L_out && R > 0) {
        std::vector<double> f = read_block<double>(h->top64, 0, (int64_t)R * R);
        for (int j = 0; j < R; ++j)
          for (int i = 0; i < R; ++i) L_out[i + (int64_t)j * R] = i >= j ? f[i + (int64_t)j * R] : 0.0;
      }
      return;
    }
    const int ne = (int)L.elim.size(), nq = (int)L.capply.size();
    if (index < 0 || index >= ne + nq) throw SgfError(SGF_EINVAL, "block index out of range");
    if (index < ne) {
      const sgf::ElimDesc& e = L.elim[index];
      const int m = e.m, k = e.k;
      const int64_t ld = (int64_t)m + k;
      info->kind = SGF_BLOCK_ELIM;
      info->cell = (int32_t)L.cell[e.cluster];
      info->m = m;
      info->k = k;
      if (!L_out && !W_out) return;
      std::vector<double> f = read_any(h, D.arena, e.front_off, ld * m);   // the first m columns
      for (int j = 0; j < m; ++j) {
        if (L_out)
          for (int i = 0; i < m; ++i) L_out[i + (int64_t)j * m] = i >= j ? f[i + j * ld] : 0.0;
        if (W_out)
          for (int q = 0; q < k; ++q) W_out[j + (int64_t)q * m] = f[(m + q) + j * ld];   // W = (rows m.. of [L; W^T])^T
      }
      return;
    }
    const sgf::CompApply& a = L.capply[index - ne];
    int ci = -1;
    for (size_t c = 0; c < L.comp.size(); ++c)
      if (L.comp[c].cf_off == a.cf_off) ci = (int)c;
    if (ci < 0) throw SgfError(SGF_EINVAL, "compressed separator not found");
    const sgf::CompDesc& d = L.comp[ci];
    const int sdim = d.s, r = L.rank[ci];
    info->kind = SGF_BLOCK_COMP;
    info->cell = (int32_t)L.cell[d.cluster];
    info->m = sdim;
    info->k = d.K;
    info->r = r;
    if (L_out) {
      const int64_t ld = (int64_t)sdim + d.K;
      std::vector<double> f = read_any(h, D.cf, d.cf_off, ld * sdim);
      for (int j = 0; j < sdim; ++j)
        for (int i = 0; i < sdim; ++i) L_out[i + (int64_t)j * sdim] = i >= j ? f[i + j * ld] : 0.0;
    }
    if (V_out || rdiag_out) {
      std::vector<double> v = read_any(h, D.nbuf, d.n_off, (int64_t)sdim * r);
      for (int j = 0; j < r; ++j) {
        if (rdiag_out) rdiag_out[j] = v[j + (int64_t)j * sdim];
        for (int i = 0; V_out && i < sdim; ++i)
          V_out[i + (int64_t)j * sdim] = i < j ? 0.0 : i == j ? 1.0 : v[i + (int64_t)j * sdim];
      }
    }
    if (tau_out) {
      std::vector<double> t = read_any(h, D.tau, d.tau_off, r);
      std::copy(t.begin(), t.end(), tau_out);
    }
  });
}

sgf_status sgf_plan_dry_run(sgf_handle h, sgf_rank_fn rank_fn, void* ctx) {
  if (!h || !rank_fn) return fail(SGF_EINVAL, "NULL argument");
  if (h->factored) return fail(SGF_ESTATE, "dry run on a factorized handle");
  return guard([&] {
    sgf::Plan& P = h->plan;
    P.levels.resize(1);
    P.parts.resize(1);
    for (size_t q = 1; q < h->lev.size(); ++q) h->lev[q].uploaded = false;
    P.max_node = 0;
    for (int s : P.levels[0].size) P.max_node = std::max<int64_t>(P.max_node, s);
    std::vector<sgf::CopyDesc> bm, pm;
    while (!P.levels.back().top) {
      sgf::Level& L = P.levels.back();
      L.rank.assign(L.comp.size(), 0);
      for (size_t c = 0; c < L.comp.size(); ++c) {
        int r = rank_fn(L.t, L.cell[L.comp[c].cluster], L.comp[c].s, ctx);
        if (r < 0 || r > std::min(L.comp[c].s, L.comp[c].c)) throw SgfError(SGF_EINVAL, "rank out of range");
        L.rank[c] = r;
      }
      sgf::plan_next_level(P, bm, pm);
    }
  });
}

sgf_status sgf_set_persistent(sgf_handle h, int32_t max_workgroups) {
  if (!h || max_workgroups < 0) return fail(SGF_EINVAL, "bad persistent-launch argument");
  h->persist_cap = max_workgroups;
  return SGF_OK;
}

sgf_status sgf_set_small_compress(sgf_handle h, int32_t enable) {
  if (!h) return fail(SGF_EINVAL, "NULL handle");
  return guard([&] {
    h->small_comp = enable != 0;
    h->small_comp_one = enable == 2;
  });
}

sgf_status sgf_set_band_elim(sgf_handle h, int32_t enable) {
  if (!h) return fail(SGF_EINVAL, "NULL handle");
  return guard([&] { h->band_elim = enable != 0; });
}

sgf_status sgf_set_pair_kernel(sgf_handle h, int32_t mode) {
  if (!h || mode < -1 || mode > 1) return fail(SGF_EINVAL, "pair kernel mode must be -1, 0 or 1");
  h->pair_mode = mode;
  return SGF_OK;
}

sgf_status sgf_set_band_apply(sgf_handle h, int32_t enable) {
  if (!h || enable < 0 || enable > 2) return fail(SGF_EINVAL, "NULL handle or mode not 0, 1, 2");
  return guard([&] {
    h->band_apply = enable != 0;
    h->band1 = enable == 1;
    h->drop_graph();
  });
}

sgf_status sgf_set_small_apply(sgf_handle h, int32_t enable) {
  if (!h || enable < 0 || enable > 1) return fail(SGF_EINVAL, "NULL handle or enable not 0 or 1");
  return guard([&] {
    h->apply1 = enable != 0;
    h->drop_graph();
  });
}

}  // extern "C"

namespace {
// Plan level 1 afresh (after the basis width or the compression changed) and
// drop every level's device state and the factor; the analysis inputs stay.
void replan(sgf_handle h) {
  h->drop_graph();
  h->lev.clear();
  h->plan.levels.clear();
  h->plan.parts.clear();
  sgf::plan_level1(h->plan, h->h_rowptr.data(), h->h_colidx.data());
  h->dev_static = false;
  h->factored = false;
  h->top_tiled = false;
  ++h->epoch;
}
}  // namespace

extern "C" {

sgf_status sgf_set_basis(sgf_handle h, int32_t ncols, const double* basis) {
  if (!h) return fail(SGF_EINVAL, "NULL handle");
  if (ncols < 0 || ncols > SGF_MAX_BASIS_COLS || (ncols > 0 && !basis))
    return fail(SGF_EINVAL, "basis: 1.." + std::to_string(SGF_MAX_BASIS_COLS) + " columns and a host array are needed");
  if (ncols == 0 && h->plan.opt.q != 0 && h->h_coords.empty())
    return fail(SGF_EINVAL, "no coordinates for the monomial basis of degree q > 0");
  return guard([&] {
    sgf::Plan& P = h->plan;
    for (int64_t i = 0; i < P.n * (int64_t)ncols; ++i)
      if (!std::isfinite(basis[i])) throw SgfError(SGF_EINVAL, "basis holds a non-finite value");
    if (ncols > 0) {
      h->h_basis.assign(basis, basis + P.n * (int64_t)ncols);
      P.pi = ncols;
    } else {
      h->h_basis.clear();
      P.pi = sgf::poly_cols(P.opt.dim, P.opt.q, P.opt.dpn);
    }
    h->d_basis.release();
    h->low_rank = false;
    h->lr_rank.clear();
    P.opt.compression = 0;
    replan(h);
  });
}

sgf_status sgf_set_low_rank(sgf_handle h, int32_t enable) {
  if (!h) return fail(SGF_EINVAL, "NULL handle");
  return guard([&] {
    sgf::Plan& P = h->plan;
    if (enable) {
      if (h->low_rank) return;
      if (!h->factored) throw SgfError(SGF_ESTATE, "low-rank mode needs a polynomial factorization to take the ranks from");
      h->lr_rank.assign(P.levels.size(), {});
      for (size_t li = 0; li + 1 < P.levels.size(); ++li) h->lr_rank[li] = P.levels[li].rank;
      h->low_rank = true;
      P.opt.compression = 1;
    } else {
      if (!h->low_rank) return;
      h->low_rank = false;
      h->lr_rank.clear();
      P.opt.compression = 0;
    }
    replan(h);
  });
}

sgf_status sgf_set_device_coarsen(sgf_handle h, int32_t enable) {
  if (!h) return fail(SGF_EINVAL, "NULL handle");
  if (enable)
    return fail(SGF_EINVAL, "the device coarsening is switched off in this build (its kernel faulted the GPU on "
                            "uploaded tables read after their host vectors were freed; fixed, not yet re-tested)");
  return guard([&] {
    if (h->device_coarsen == (enable != 0)) return;
    h->device_coarsen = enable != 0;
    replan(h);
  });
}

sgf_status sgf_set_apply_graph(sgf_handle h, int32_t enable) {
  if (!h) return fail(SGF_EINVAL, "NULL handle");
  return guard([&] { h->use_graph = enable != 0; });
}

sgf_status sgf_profile_select(sgf_handle h, const char* kernel_class) {
  if (!h) return fail(SGF_EINVAL, "NULL handle");
  return guard([&] { h->prof.only = kernel_class ? kernel_class : ""; });
}

sgf_status sgf_profile_enable(sgf_handle h, int32_t enable) {
  if (!h) return fail(SGF_EINVAL, "NULL handle");
  return guard([&] {
    h->prof.drain();
    h->prof.stats.clear();
    h->prof.on = enable != 0;
  });
}

sgf_status sgf_profile_read(sgf_handle h, sgf_kernel_stat* out, int32_t cap, int32_t* count) {
  if (!h || !count) return fail(SGF_EINVAL, "NULL argument");
  return guard([&] {
    h->prof.drain();
    *count = (int32_t)h->prof.stats.size();
    for (int i = 0; i < std::min<int>(cap, (int)h->prof.stats.size()); ++i) out[i] = h->prof.stats[i];
  });
}

sgf_status sgf_destroy(sgf_handle h) {
  delete h;
  return SGF_OK;
}

}  // extern "C"
