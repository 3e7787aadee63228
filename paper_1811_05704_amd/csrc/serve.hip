// Serving: a request loop over many independent linear systems with
// continuous batching (C ABI amg_server_* in include/amg.h).
//
// Section 3 of the paper: the hierarchy depends only on the matrix, is set
// up once and then lives on the backend for the solve.  Here each request
// (matrix + right-hand side) is set up by a worker thread (its data-parallel
// steps on the device on the worker's own stream, with temporaries drawn from
// the budget), placed in a device memory pool under an HBM budget, and
// admitted into a slot of the live set at an iteration boundary.  One step launches a captured hipGraph of
// `check_every` Krylov iterations in which every kernel is a persistent,
// descriptor-driven launch covering the same operation of all live solves (the
// outer SpMV of every solve, then the level-1 pre-sweeps of every solve, ...).
// Converged solves are retired after the step and their slots and memory
// reused.  Each batched block reproduces the single-solve block exactly, so a
// request's result is bitwise the same alone, in any mix, and from amg_solve.

#include <algorithm>
#include <condition_variable>
#include <deque>
#include <exception>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>

#include "galerkin.hpp"
#include "solver.hpp"

namespace amg {
namespace {

constexpr int kMaxLevels = 8;        // levels per served hierarchy
constexpr int kSpmvGrid = 2048;      // persistent grid of the batched SpMV
constexpr int kVecGrid = 2048;       // persistent grid of the batched vector kernels
constexpr int kFinGrid = 64;         // one workgroup per solve
constexpr int kGemvGrid = 1024;

// ------------------------------------------------------------------ device memory pool

// First-fit allocator over one device allocation of the HBM budget; requests'
// hierarchies and vectors are carved from it so that admissions never call
// hipMalloc while other solves run.
class DevicePool {
 public:
  explicit DevicePool(size_t bytes) : size_(bytes) {
    hipError_t e = hipMalloc(&base_, bytes);
    if (e != hipSuccess || !base_) {
      (void)hipGetLastError();
      throw DevError{-5, "cannot reserve the serving pool of " + std::to_string(bytes) + " bytes"};
    }
    free_[0] = bytes;
  }
  ~DevicePool() {
    if (base_) (void)hipFree(base_);
  }
  void* alloc(size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    std::lock_guard<std::mutex> lk(mu_);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const size_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > bytes) free_[off + bytes] = len - bytes;
        used_[off] = bytes;
        in_use_ += bytes;
        return static_cast<char*>(base_) + off;
      }
    }
    return nullptr;
  }
  void free(void* p) {
    std::lock_guard<std::mutex> lk(mu_);
    const size_t off = static_cast<char*>(p) - static_cast<char*>(base_);
    auto u = used_.find(off);
    if (u == used_.end()) return;
    size_t len = u->second;
    used_.erase(u);
    in_use_ -= len;
    size_t start = off;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && next->first == off + len) {
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == start) {
        start = prev->first;
        len += prev->second;
        free_.erase(prev);
      }
    }
    free_[start] = len;
  }
  size_t in_use() {
    std::lock_guard<std::mutex> lk(mu_);
    return in_use_;
  }
  size_t size() const { return size_; }

  static void* alloc_cb(size_t bytes, void*, void* ctx) { return static_cast<DevicePool*>(ctx)->alloc(bytes); }
  static void free_cb(void* p, void*, void* ctx) { static_cast<DevicePool*>(ctx)->free(p); }

 private:
  void* base_ = nullptr;
  size_t size_;
  std::mutex mu_;
  std::map<size_t, size_t> free_;   // offset -> length
  std::unordered_map<size_t, size_t> used_;
  size_t in_use_ = 0;
};

// Device bytes a request will occupy (hierarchy in the V-cycle's precision,
// the FP64 fine matrix, dense coarse inverse, vectors, partials), rounded up
// per allocation; used to reject requests that can never fit.
// Device bytes held only during setup: the coarse matrix in CSR form, its
// dense LU factors and pivots.
size_t coarse_transient(const HostHierarchy& H) {
  const Csr& AL = H.levels.back().A;
  const size_t nL = AL.rows;
  return nL * nL * 8 + nL * 24 + (nL + 1) * 4 + static_cast<size_t>(AL.nnz()) * 12 + 10 * 256;
}

size_t footprint(const HostHierarchy& H, const amg_params& p) {
  const size_t vs = p.precision == AMG_MIXED ? 4 : 8;
  // row pointers, columns, values, the stream schedule (at most one block per
  // row) and the allocator's rounding
  auto csr = [&](const Csr& M, size_t v) { return (M.rows + 1) * 4 + M.nnz() * (4 + v) + (M.rows + 2) * 4 + 1024; };
  size_t b = 0;
  const HostLevel& f = H.levels[0];
  b += csr(f.A, 8);
  for (size_t l = 0; l + 1 < H.levels.size(); ++l) {
    const HostLevel& L = H.levels[l];
    if (l > 0) b += csr(L.A, vs);
    else if (p.precision == AMG_MIXED) b += L.A.nnz() * vs + (L.A.rows + 2) * 4 + 512;  // pattern shared with the FP64 copy
    b += csr(L.P, vs) + csr(L.R, vs);
    b += L.A.rows * vs * 7;
    if (l == 0) b += L.A.nnz() * vs + 4096;  // A diag(m) values of level 1
  }
  const size_t nL = H.levels.back().A.rows;
  b += nL * nL * 8 + nL * 64;
  b += coarse_transient(H);  // LU factors while the coarse inverse is formed
  b += f.A.rows * 8 * 16;  // Krylov vectors and partials
  return b + 64 * 256;
}

// ------------------------------------------------------------------ iteration descriptors

template <class T>
struct IterDesc {
  Batch<SpmvItem<double, GatherX<double, double>, EpiStoreDot>> outer;
  Batch<FinItem> fin_alpha;
  Batch<UpdItem> update;
  Batch<FinItem> fin_rr;
  Batch<SpmvItem<T, GatherX<T, double>, EpiResid<T, double>>> pre0;
  Batch<SpmvItem<T, GatherX<T, T>, EpiResid<T, T>>> pre[kMaxLevels];
  Batch<SpmvItem<T, GatherX<T, T>, EpiRestrict<T>>> restrict_mid[kMaxLevels];
  Batch<SpmvItem<T, GatherX<T, T>, EpiStore<T, T>>> restrict_last[kMaxLevels];
  Batch<GemvItem<T>> coarse;
  Batch<SpmvItem<T, GatherX<T, T>, EpiProlong<T, double, 1>>> prolong0;
  Batch<SpmvItem<T, GatherX<T, T>, EpiProlong<T, T, 2>>> prolong[kMaxLevels];
  Batch<SpmvItem<T, GatherX<T, T>, EpiSmooth<T, double, double, 1>>> post0;
  Batch<SpmvItem<T, GatherX<T, T>, EpiSmooth<T, T, T, 0>>> post[kMaxLevels];
  Batch<FinItem> fin_rho;
  Batch<DirItem> dir;
};

template <class Item>
void batch_clear(Batch<Item>& b) {
  b.n = 0;
  b.total = 0;
  b.off[0] = 0;
}

template <class Item>
void batch_add(Batch<Item>& b, const Item& it, int blocks) {
  b.it[b.n] = it;
  b.off[b.n + 1] = b.off[b.n] + blocks;
  b.total = b.off[b.n + 1];
  b.n += 1;
}

// Descriptor of one solve's SpMV in a batch.  The batched kernel dispatches
// the stream schedule (block table, (lanes, block class) of the single-solve
// switch) and the vector schedule (matrices of mean row length above 512);
// anything else is refused here, on the host, before it could reach a launch.
template <class T, class G, class E>
SpmvItem<T, G, E> spmv_item(const DevCsr<T>& M, G g, E e, double* partials, const int* skip) {
  if (M.rows > 0) {
    if (M.kind == 0 && (!M.blk || !stream_dispatchable(M.lanes, M.bclass)))
      throw DevError{-6, "served matrix has a stream schedule the batched kernel cannot run"};
    if (M.kind == 1 && M.lanes != 64)
      throw DevError{-6, "served matrix has a vector schedule the batched kernel cannot run"};
    if (M.kind != 0 && M.kind != 1) throw DevError{-6, "served matrix has an unknown SpMV schedule"};
  }
  return SpmvItem<T, G, E>{M.view(), g, e, partials, skip, M.kind, M.lanes, M.bclass};
}

template <class T, class G, class E>
void launch_batch(const Batch<SpmvItem<T, G, E>>* b, hipStream_t s) {
  batched_spmv_kernel<T, G, E><<<kSpmvGrid, kBS, 0, s>>>(b);
  AMG_LAUNCHED();
}

template <class T>
DevHierarchy<T>& hier(amg_solver& S);
template <>
DevHierarchy<double>& hier<double>(amg_solver& S) { return S.h64; }
template <>
DevHierarchy<float>& hier<float>(amg_solver& S) { return S.h32; }

// ------------------------------------------------------------------ requests

struct Request {
  uint64_t id = 0;
  Csr A;
  std::vector<double> f;
  std::unique_ptr<amg_solver> S;
  int status = 0;
  std::vector<double> x;
  amg_info info{};
  double t_submit = 0, t_ready = 0, t_admit = 0, t_done = 0;
  int restarts = 0;
  std::string error;  // what failed, for a request with status < 0
  int slot = -1;
  size_t reserved = 0;  // bytes of the budget held for this request
};

}  // namespace
}  // namespace amg

struct amg_server_s {
  amg_params prm{};
  int device = 0;
  int max_slots = 0;
  hipStream_t stream = nullptr;      // batched compute
  hipStream_t cap_stream = nullptr;  // graph capture
  std::unique_ptr<amg::DevicePool> pool;
  amg_allocator alloc{};

  std::mutex mu;
  std::condition_variable cv_work, cv_mem, cv_ready;
  std::deque<amg::Request*> pending, ready, finished;
  std::vector<std::thread> workers;
  bool stopping = false;
  int setting_up = 0;
  size_t reserved = 0;  // budget bytes held by requests being placed, waiting or live

  std::vector<amg::Request*> slots;
  amg::KState* states = nullptr;        // device, one per slot
  amg::KState* states_host = nullptr;   // pinned poll target
  amg::KState* states_init = nullptr;   // pinned staging for admissions
  void* desc_dev = nullptr;
  void* desc_host = nullptr;
  size_t desc_bytes = 0;
  bool dirty = true;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_depth = 0;
  int64_t completed = 0;

  ~amg_server_s();
};

namespace amg {
namespace {

template <class T>
void build_desc(amg_server_s& V, IterDesc<T>& D) {
  batch_clear(D.outer);
  batch_clear(D.fin_alpha);
  batch_clear(D.update);
  batch_clear(D.fin_rr);
  batch_clear(D.pre0);
  batch_clear(D.coarse);
  batch_clear(D.prolong0);
  batch_clear(D.post0);
  batch_clear(D.fin_rho);
  batch_clear(D.dir);
  for (int l = 0; l < kMaxLevels; ++l) {
    batch_clear(D.pre[l]);
    batch_clear(D.restrict_mid[l]);
    batch_clear(D.restrict_last[l]);
    batch_clear(D.prolong[l]);
    batch_clear(D.post[l]);
  }
  for (Request* q : V.slots) {
    if (!q) continue;
    amg_solver& S = *q->S;
    const int n = static_cast<int>(S.n);
    const int vb = vec_blocks(n);
    const int* skip = &S.st->done;
    batch_add(D.outer, spmv_item(S.A0, GatherX<double, double>{S.p}, EpiStoreDot{S.q, S.p}, S.partials, skip),
              S.A0.nblocks);
    batch_add(D.fin_alpha, FinItem{S.partials, S.A0.nblocks, S.st}, 1);
    batch_add(D.update, UpdItem{n, S.x, S.r, S.p, S.q, S.st, S.partials}, vb);
    batch_add(D.fin_rr, FinItem{S.partials, vb, S.st}, 1);
    DevHierarchy<T>& H = hier<T>(S);
    const int L = static_cast<int>(H.lev.size()) + 1;
    if (L == 1) throw DevError{-1, "served systems need at least two levels"};
    for (int l = 0; l < L - 1; ++l) {
      DevLevel<T>& lv = H.lev[l];
      DevLevel<T>* next = (l + 1 < L - 1) ? &H.lev[l + 1] : nullptr;
      if (l == 0)
        batch_add(D.pre0, spmv_item(lv.As, GatherX<T, double>{S.r}, EpiResid<T, double>{lv.r, S.r}, nullptr, skip),
                  lv.A.nblocks);
      else
        batch_add(D.pre[l], spmv_item(lv.A, GatherX<T, T>{lv.mf}, EpiResid<T, T>{lv.r, lv.f}, nullptr, skip),
                  lv.A.nblocks);
      if (next)
        batch_add(D.restrict_mid[l],
                  spmv_item(lv.R, GatherX<T, T>{lv.r}, EpiRestrict<T>{next->f, next->mf, next->m}, nullptr, skip),
                  lv.R.nblocks);
      else
        batch_add(D.restrict_last[l], spmv_item(lv.R, GatherX<T, T>{lv.r}, EpiStore<T, T>{H.fL}, nullptr, skip),
                  lv.R.nblocks);
      const T* zc = next ? next->z : H.zL;
      if (l == 0) {
        batch_add(D.prolong0,
                  spmv_item(lv.P, GatherX<T, T>{zc}, EpiProlong<T, double, 1>{lv.y, lv.m, S.r, nullptr}, nullptr, skip),
                  lv.P.nblocks);
        batch_add(D.post0,
                  spmv_item(lv.A, GatherX<T, T>{lv.y}, EpiSmooth<T, double, double, 1>{S.z, lv.y, lv.m, S.r},
                            S.partials, skip),
                  lv.A.nblocks);
      } else {
        batch_add(D.prolong[l],
                  spmv_item(lv.P, GatherX<T, T>{zc}, EpiProlong<T, T, 2>{lv.y, lv.m, lv.f, lv.mf}, nullptr, skip),
                  lv.P.nblocks);
        batch_add(D.post[l],
                  spmv_item(lv.A, GatherX<T, T>{lv.y}, EpiSmooth<T, T, T, 0>{lv.z, lv.y, lv.m, lv.f}, nullptr, skip),
                  lv.A.nblocks);
      }
    }
    batch_add(D.coarse, GemvItem<T>{S.nL, S.Ainv, H.fL, H.zL, skip}, S.nL);
    batch_add(D.fin_rho, FinItem{S.partials, H.lev[0].A.nblocks, S.st}, 1);
    batch_add(D.dir, DirItem{n, S.p, S.z, S.st}, vb);
  }
}

// One batched PCG iteration over every live solve (same kernel order as the
// single-solve iteration).
template <class T>
void enqueue_batched_iteration(const IterDesc<T>* D, int depth, hipStream_t s) {
  launch_batch(&D->outer, s);
  batched_finalize_kernel<1><<<kFinGrid, kFinBS, 0, s>>>(&D->fin_alpha, kFinAlpha);
  batched_update_kernel<<<kVecGrid, kVecBS, 0, s>>>(&D->update);
  batched_finalize_kernel<1><<<kFinGrid, kFinBS, 0, s>>>(&D->fin_rr, kFinPcgRR);
  AMG_LAUNCHED();
  launch_batch(&D->pre0, s);
  for (int l = 0; l < depth - 1; ++l) {
    if (l > 0) launch_batch(&D->pre[l], s);
    launch_batch(&D->restrict_mid[l], s);
    launch_batch(&D->restrict_last[l], s);
  }
  batched_gemv_kernel<T><<<kGemvGrid, kBS, 0, s>>>(&D->coarse);
  AMG_LAUNCHED();
  for (int l = depth - 2; l >= 1; --l) {
    launch_batch(&D->prolong[l], s);
    launch_batch(&D->post[l], s);
  }
  launch_batch(&D->prolong0, s);
  launch_batch(&D->post0, s);
  batched_finalize_kernel<1><<<kFinGrid, kFinBS, 0, s>>>(&D->fin_rho, kFinPcgRho);
  batched_dir_kernel<<<kVecGrid, kVecBS, 0, s>>>(&D->dir);
  AMG_LAUNCHED();
}

// Graph of check_every batched iterations over hierarchies of up to `depth`
// levels; re-captured when the deepest live hierarchy changes.
template <class T>
void capture_graph(amg_server_s& V, int depth) {
  if (V.exec && V.graph_depth == depth) return;
  if (V.exec) (void)hipGraphExecDestroy(V.exec);
  if (V.graph) (void)hipGraphDestroy(V.graph);
  V.exec = nullptr;
  V.graph = nullptr;
  const IterDesc<T>* D = static_cast<const IterDesc<T>*>(V.desc_dev);
  AMG_HIP(hipStreamBeginCapture(V.cap_stream, hipStreamCaptureModeThreadLocal));
  try {
    for (int it = 0; it < V.prm.check_every; ++it) enqueue_batched_iteration<T>(D, depth, V.cap_stream);
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(V.cap_stream, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  AMG_HIP(hipStreamEndCapture(V.cap_stream, &V.graph));
  AMG_HIP(hipGraphInstantiate(&V.exec, V.graph, nullptr, nullptr, 0));
  V.graph_depth = depth;
}

// Host worker: build the hierarchy, place it in the pool, upload f.
// Allocator for setup temporaries (the device setup steps): memory from the
// pool, reserved against the budget without waiting.  An allocation that the
// unreserved budget cannot cover fails at once, and that step then runs on
// the host; so no worker waits for memory while holding some.  (Holding the
// temporaries to a share of the budget was measured to slow serving: more
// steps then run on the host.)
class TransientAlloc {
 public:
  explicit TransientAlloc(amg_server_s* V) : V_(V) {}
  amg_allocator handle() { return amg_allocator{&TransientAlloc::alloc_cb, &TransientAlloc::free_cb, this}; }

 private:
  static void* alloc_cb(size_t bytes, void*, void* ctx) {
    auto* t = static_cast<TransientAlloc*>(ctx);
    amg_server_s* V = t->V_;
    bytes = (bytes + 255) & ~size_t(255);
    {
      std::lock_guard<std::mutex> lk(V->mu);
      if (V->reserved + bytes > V->pool->size()) return nullptr;
      V->reserved += bytes;
    }
    void* p = V->pool->alloc(bytes);
    if (!p) {
      t->release(bytes);
      return nullptr;
    }
    t->sizes_[p] = bytes;
    return p;
  }
  static void free_cb(void* p, void*, void* ctx) {
    auto* t = static_cast<TransientAlloc*>(ctx);
    auto it = t->sizes_.find(p);
    if (it == t->sizes_.end()) return;
    const size_t bytes = it->second;
    t->sizes_.erase(it);
    t->V_->pool->free(p);
    t->release(bytes);
  }
  void release(size_t bytes) {
    {
      std::lock_guard<std::mutex> lk(V_->mu);
      V_->reserved -= bytes;
    }
    V_->cv_mem.notify_all();
  }
  amg_server_s* V_;
  std::unordered_map<void*, size_t> sizes_;  // used by one worker thread only
};

void worker_main(amg_server_s* V, int threads) {
  set_setup_threads(threads);
  (void)hipSetDevice(V->device);
  hipStream_t ws = nullptr;
  rocblas_handle blas = nullptr;
  bool blas_ok = false;
  if (hipStreamCreateWithFlags(&ws, hipStreamNonBlocking) == hipSuccess) {
    auto lk = blas_lock();
    blas_ok = rocblas_create_handle(&blas) == rocblas_status_success;
  }
  if (!blas_ok) {
    std::lock_guard<std::mutex> lk(V->mu);
    V->stopping = true;
    V->cv_work.notify_all();
    return;
  }
  for (;;) {
    Request* q = nullptr;
    {
      std::unique_lock<std::mutex> lk(V->mu);
      V->cv_work.wait(lk, [&] { return V->stopping || !V->pending.empty(); });
      if (V->stopping) break;
      q = V->pending.front();
      V->pending.pop_front();
      V->setting_up += 1;
    }
    const double t0 = now_s();
    try {
      q->S = std::make_unique<amg_solver>();
      amg_solver& S = *q->S;
      S.prm = V->prm;
      TransientAlloc scratch(V);
      const amg_allocator scratch_alloc = scratch.handle();
      std::unique_ptr<SetupAccel> accel = make_device_setup_accel(&scratch_alloc, ws);
      S.host = build_hierarchy(std::move(q->A), setup_params(V->prm), accel.get());
      accel.reset();  // its device memory goes back to the budget
      if (S.host.levels.size() < 2) throw SetupError{-1, "served systems need at least two levels"};
      if (S.host.levels.size() > static_cast<size_t>(kMaxLevels))
        throw SetupError{-8, "hierarchy deeper than the serving limit"};
      const size_t need = footprint(S.host, V->prm);
      if (need > V->pool->size()) throw SetupError{-5, "request does not fit in the HBM budget"};
      {
        // Admission by footprint: hold `need` bytes of the budget before placing.
        std::unique_lock<std::mutex> lk(V->mu);
        V->cv_mem.wait(lk, [&] { return V->stopping || V->reserved + need <= V->pool->size(); });
        if (V->stopping) throw DevError{-5, "server stopping"};
        V->reserved += need;
        q->reserved = need;
      }
      DeviceSetupOpts opts;
      opts.standalone = false;
      opts.blas = blas;
      for (bool failed_alone = false;;) {
        try {
          device_setup(S, &V->alloc, ws, opts);
          break;
        } catch (const DevError& e) {
          if (e.code != -5) throw;
          drop_device_state(S);  // give back what was taken, wait for retirements
          std::unique_lock<std::mutex> lk(V->mu);
          if (V->reserved == q->reserved) {
            // Alone in the pool: the memory in the way may have belonged to
            // another worker's setup that finished meanwhile (its temporaries
            // come and go), so try once more; failing again alone, it cannot fit.
            if (failed_alone) throw;
            failed_alone = true;
            continue;
          }
          failed_alone = false;
          V->cv_mem.wait_for(lk, std::chrono::milliseconds(20));
          if (V->stopping) throw DevError{-5, "server stopping"};
        }
      }
      AMG_HIP(hipMemcpyAsync(S.f, q->f.data(), sizeof(double) * S.n, hipMemcpyHostToDevice, ws));
      AMG_HIP(hipStreamSynchronize(ws));
      {
        // the coarse LU factors are gone: hand their share of the budget back
        const size_t t = std::min(coarse_transient(S.host), q->reserved);
        std::lock_guard<std::mutex> lk(V->mu);
        V->reserved -= t;
        q->reserved -= t;
      }
      V->cv_mem.notify_all();
      S.arena->set_stream(V->stream);  // from now on the solve lives on the server's stream
      S.setup_s = now_s() - t0;
      q->t_ready = now_s();
      std::lock_guard<std::mutex> lk(V->mu);
      V->setting_up -= 1;
      V->ready.push_back(q);
      V->cv_ready.notify_all();
    } catch (const SetupError& e) {
      q->status = e.code;
      q->error = e.msg;
    } catch (const DevError& e) {
      q->status = e.code;
      q->error = e.msg;
    } catch (const std::bad_alloc&) {
      q->status = AMG_ERR_OOM;
      q->error = "host memory exhausted in the setup worker";
    } catch (const std::exception& e) {
      q->status = AMG_ERR_INVALID_ARG;
      q->error = e.what();
    } catch (...) {
      q->status = AMG_ERR_INVALID_ARG;
      q->error = "unknown error in the setup worker";
    }
    if (q->status != 0) {
      if (q->S) q->S.reset();
      q->t_done = now_s();
      std::lock_guard<std::mutex> lk(V->mu);
      V->reserved -= q->reserved;
      q->reserved = 0;
      V->setting_up -= 1;
      V->finished.push_back(q);
      V->cv_mem.notify_all();
      V->cv_ready.notify_all();
    }
  }
  if (blas) {
    auto lk = blas_lock();
    rocblas_destroy_handle(blas);
  }
  if (ws) (void)hipStreamDestroy(ws);
}

// Admit ready requests into free slots: initial residual, first V-cycle and
// search direction with the single-solve kernels.
void admit(amg_server_s& V) {
  for (int slot = 0; slot < V.max_slots; ++slot) {
    if (V.slots[slot]) continue;
    Request* q = nullptr;
    {
      std::lock_guard<std::mutex> lk(V.mu);
      if (V.ready.empty()) return;
      q = V.ready.front();
      V.ready.pop_front();
    }
    amg_solver& S = *q->S;
    S.st = V.states + slot;
    KState init{};
    init.tol = V.prm.tol;
    init.max_iter = V.prm.max_iter;
    init.first = 1;
    V.states_init[slot] = init;
    AMG_HIP(hipMemcpyAsync(S.st, V.states_init + slot, sizeof(KState), hipMemcpyHostToDevice, V.stream));
    fill_kernel<double><<<vec_blocks(S.n), kVecBS, 0, V.stream>>>(static_cast<int>(S.n), S.x, 0.0);
    AMG_LAUNCHED();
    enqueue_pcg_start(S, V.stream);
    q->slot = slot;
    q->t_admit = now_s();
    V.slots[slot] = q;
    V.dirty = true;
  }
}

void retire(amg_server_s& V) {
  // Which live solves stopped?
  std::vector<int> done;
  for (int slot = 0; slot < V.max_slots; ++slot)
    if (V.slots[slot] && V.states_host[slot].done != kRunning) done.push_back(slot);
  if (done.empty()) return;
  // True residual of each (same kernels as amg_solve).
  for (int slot : done) {
    amg_solver& S = *V.slots[slot]->S;
    if (V.states_host[slot].done == kZeroRhs) continue;
    int nb = launch_spmv(S.A0, GatherX<double, double>{S.x}, EpiResidNorms{S.tmp, S.f}, S.partials, nullptr, V.stream);
    fin(S, 2, nb, kFinTrue, V.stream);
  }
  AMG_HIP(hipMemcpyAsync(V.states_host, V.states, sizeof(KState) * V.max_slots, hipMemcpyDeviceToHost, V.stream));
  AMG_HIP(hipStreamSynchronize(V.stream));
  for (int slot : done) {
    Request* q = V.slots[slot];
    amg_solver& S = *q->S;
    const KState k = V.states_host[slot];
    if (k.done == kConverged && k.true_rr > k.tol2 && q->restarts == 0) {
      q->restarts += 1;  // restart once from the current iterate (stays live)
      enqueue_pcg_start(S, V.stream);
      continue;
    }
    if (k.done == kZeroRhs) {
      fill_kernel<double><<<vec_blocks(S.n), kVecBS, 0, V.stream>>>(static_cast<int>(S.n), S.x, 0.0);
      AMG_LAUNCHED();
    }
    q->x.resize(S.n);
    AMG_HIP(hipMemcpyAsync(q->x.data(), S.x, sizeof(double) * S.n, hipMemcpyDeviceToHost, V.stream));
    AMG_HIP(hipStreamSynchronize(V.stream));
    int status = AMG_OK;
    switch (k.done) {
      case kConverged: status = (k.true_rr <= k.tol2) ? AMG_OK : AMG_NOT_CONVERGED; break;
      case kZeroRhs: status = AMG_OK; break;
      case kMaxIter: status = AMG_NOT_CONVERGED; break;
      case kBreakdown: status = AMG_ERR_BREAKDOWN; break;
      default: status = AMG_ERR_NAN; break;
    }
    q->status = status;
    q->t_done = now_s();
    amg_info& in = q->info;
    in.iters = k.iters;
    in.levels = static_cast<int32_t>(S.host.levels.size());
    in.restarts = q->restarts;
    in.status = status;
    const bool zero = (k.done == kZeroRhs);
    in.rel_resid = zero ? 0.0 : std::sqrt(k.rr / k.ff);
    in.true_rel_resid = zero ? 0.0 : std::sqrt(k.true_rr / k.ff);
    in.setup_s = S.setup_s;
    in.solve_s = q->t_done - q->t_admit;
    double nnz = 0;
    for (auto& lv : S.host.levels) nnz += double(lv.A.nnz());
    in.op_complexity = nnz / double(S.host.levels[0].A.nnz());
    q->S.reset();  // device memory back to the pool
    V.slots[slot] = nullptr;
    V.dirty = true;
    std::lock_guard<std::mutex> lk(V.mu);
    V.reserved -= q->reserved;
    q->reserved = 0;
    V.finished.push_back(q);
    V.completed += 1;
    V.cv_mem.notify_all();
  }
}

template <class T>
void server_step(amg_server_s& V) {
  admit(V);
  int live = 0;
  for (Request* q : V.slots) live += q != nullptr;
  if (live > 0) {
    if (V.dirty) {
      build_desc<T>(V, *static_cast<IterDesc<T>*>(V.desc_host));
      AMG_HIP(hipMemcpyAsync(V.desc_dev, V.desc_host, V.desc_bytes, hipMemcpyHostToDevice, V.stream));
      int depth = 2;
      for (Request* q : V.slots)
        if (q) depth = std::max(depth, static_cast<int>(q->S->host.levels.size()));
      capture_graph<T>(V, depth);
      V.dirty = false;
    }
    AMG_HIP(hipGraphLaunch(V.exec, V.stream));
  }
  AMG_HIP(hipMemcpyAsync(V.states_host, V.states, sizeof(KState) * V.max_slots, hipMemcpyDeviceToHost, V.stream));
  AMG_HIP(hipStreamSynchronize(V.stream));
  retire(V);
}

}  // namespace
}  // namespace amg

amg_server_s::~amg_server_s() {
  {
    std::lock_guard<std::mutex> lk(mu);
    stopping = true;
  }
  cv_work.notify_all();
  cv_mem.notify_all();
  cv_ready.notify_all();
  for (auto& t : workers) t.join();
  if (stream) (void)hipStreamSynchronize(stream);
  for (auto* q : slots) delete q;
  for (auto* q : pending) delete q;
  for (auto* q : ready) delete q;
  for (auto* q : finished) delete q;
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (states_host) (void)hipHostFree(states_host);
  if (states_init) (void)hipHostFree(states_init);
  if (desc_host) (void)hipHostFree(desc_host);
  if (desc_dev) (void)hipFree(desc_dev);
  if (states) (void)hipFree(states);
  pool.reset();
  if (cap_stream) (void)hipStreamDestroy(cap_stream);
}

using namespace amg;

extern "C" {

amg_status amg_server_create(const amg_params* p, size_t hbm_budget_bytes, int32_t max_slots, int32_t setup_threads,
                             void* hip_stream, amg_server* out) {
  if (out) *out = nullptr;
  return guarded([&]() -> amg_status {
    if (!out) throw SetupError{-1, "out must not be NULL"};
    if (max_slots < 1 || max_slots > kMaxSlots) throw SetupError{-1, "max_slots must be in [1, 64]"};
    if (setup_threads < 1 || setup_threads > 64) throw SetupError{-1, "setup_threads must be in [1, 64]"};
    if (hbm_budget_bytes < (size_t(1) << 20)) throw SetupError{-1, "HBM budget below 1 MiB"};
    auto V = std::make_unique<amg_server_s>();
    if (p) V->prm = *p;
    else amg_params_default(&V->prm);
    check_params(V->prm);
    if (V->prm.solver != AMG_CG || V->prm.npre != 1 || V->prm.npost != 1 || V->prm.relax == AMG_CHEBYSHEV)
      throw SetupError{-1, "serving runs PCG with one pre- and one post-sweep of SPAI-0 or Jacobi"};
    AMG_HIP(hipGetDevice(&V->device));
    V->max_slots = max_slots;
    V->stream = static_cast<hipStream_t>(hip_stream);
    V->pool = std::make_unique<DevicePool>(hbm_budget_bytes);
    V->alloc = amg_allocator{&DevicePool::alloc_cb, &DevicePool::free_cb, V->pool.get()};
    V->slots.assign(max_slots, nullptr);
    AMG_HIP(hipMalloc(reinterpret_cast<void**>(&V->states), sizeof(KState) * max_slots));
    AMG_HIP(hipHostMalloc(reinterpret_cast<void**>(&V->states_host), sizeof(KState) * max_slots, hipHostMallocDefault));
    AMG_HIP(hipHostMalloc(reinterpret_cast<void**>(&V->states_init), sizeof(KState) * max_slots, hipHostMallocDefault));
    V->desc_bytes = V->prm.precision == AMG_MIXED ? sizeof(IterDesc<float>) : sizeof(IterDesc<double>);
    AMG_HIP(hipMalloc(&V->desc_dev, V->desc_bytes));
    AMG_HIP(hipHostMalloc(&V->desc_host, V->desc_bytes, hipHostMallocDefault));
    std::memset(V->desc_host, 0, V->desc_bytes);
    for (int i = 0; i < max_slots; ++i) {
      KState k{};
      k.done = kConverged;
      V->states_host[i] = k;
    }
    // Empty batches (n = 0) until the first admission.
    AMG_HIP(hipMemcpyAsync(V->desc_dev, V->desc_host, V->desc_bytes, hipMemcpyHostToDevice, V->stream));
    AMG_HIP(hipMemcpyAsync(V->states, V->states_host, sizeof(KState) * max_slots, hipMemcpyHostToDevice, V->stream));
    AMG_HIP(hipStreamSynchronize(V->stream));
    AMG_HIP(hipStreamCreateWithFlags(&V->cap_stream, hipStreamNonBlocking));
    for (int t = 0; t < setup_threads; ++t) V->workers.emplace_back(worker_main, V.get(), 1);
    *out = V.release();
    return AMG_OK;
  });
}

amg_status amg_server_submit(amg_server s, uint64_t request_id, int64_t n, const int64_t* row_ptr, const int32_t* col,
                             const double* val, const double* f_host) {
  return guarded([&]() -> amg_status {
    if (!s || !f_host) throw SetupError{-1, "NULL argument"};
    // the client's thread: no helper threads beside the workers and the driver
    ScopedSetupThreads one(1);
    validate_csr(n, row_ptr, col, val);
    auto q = std::make_unique<Request>();
    q->id = request_id;
    q->A = to_csr(n, row_ptr, col, val);
    q->f.assign(f_host, f_host + n);
    q->t_submit = now_s();
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) throw DevError{-6, "server stopped (a worker failed to start)"};
    s->pending.push_back(q.release());
    s->cv_work.notify_one();
    return AMG_OK;
  });
}

amg_status amg_server_step(amg_server s, int32_t* live, int32_t* waiting) {
  return guarded([&]() -> amg_status {
    if (!s) throw SetupError{-1, "NULL server"};
    if (s->prm.precision == AMG_MIXED) server_step<float>(*s);
    else server_step<double>(*s);
    int nl = 0;
    for (auto* q : s->slots) nl += q != nullptr;
    if (live) *live = nl;
    if (waiting) {
      std::lock_guard<std::mutex> lk(s->mu);
      *waiting = static_cast<int32_t>(s->pending.size() + s->ready.size()) + s->setting_up;
    }
    return AMG_OK;
  });
}

amg_status amg_server_wait_ready(amg_server s, int32_t count, double timeout_s, int32_t* ready) {
  return guarded([&]() -> amg_status {
    if (!s || count < 0 || !(timeout_s >= 0.0)) throw SetupError{-1, "bad argument"};
    std::unique_lock<std::mutex> lk(s->mu);
    const auto deadline = std::chrono::steady_clock::now() + std::chrono::duration<double>(timeout_s);
    while (static_cast<int32_t>(s->ready.size()) < count &&
           !(s->pending.empty() && s->setting_up == 0)) {
      if (s->cv_ready.wait_until(lk, deadline) == std::cv_status::timeout) break;
    }
    if (ready) *ready = static_cast<int32_t>(s->ready.size());
    return static_cast<int32_t>(s->ready.size()) >= count ? AMG_OK : AMG_NOT_CONVERGED;
  });
}

amg_status amg_server_poll(amg_server s, uint64_t* request_id, int64_t* n) {
  return guarded([&]() -> amg_status {
    if (!s || !request_id || !n) throw SetupError{-1, "NULL argument"};
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->finished.empty()) return AMG_NOT_CONVERGED;  // 1: nothing ready
    *request_id = s->finished.front()->id;
    *n = static_cast<int64_t>(s->finished.front()->x.size());
    return AMG_OK;
  });
}

amg_status amg_server_fetch(amg_server s, uint64_t request_id, double* x_host, amg_info* info, double* times) {
  return guarded([&]() -> amg_status {
    if (!s) throw SetupError{-1, "NULL server"};
    Request* q = nullptr;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      if (s->finished.empty() || s->finished.front()->id != request_id)
        throw SetupError{-1, "request is not the next finished one"};
      q = s->finished.front();
      s->finished.pop_front();
    }
    std::unique_ptr<Request> own(q);
    if (x_host && !q->x.empty()) std::memcpy(x_host, q->x.data(), sizeof(double) * q->x.size());
    if (info) *info = q->info;
    if (times) {
      times[0] = q->t_submit;
      times[1] = q->t_ready;
      times[2] = q->t_admit;
      times[3] = q->t_done;
    }
    if (q->status < 0)
      g_last_error = "request failed with status " + std::to_string(q->status) + (q->error.empty() ? "" : ": " + q->error);
    return static_cast<amg_status>(q->status);
  });
}

void amg_server_destroy(amg_server s) { delete s; }

}  // extern "C"
