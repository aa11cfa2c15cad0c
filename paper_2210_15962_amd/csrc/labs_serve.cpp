// labs_serve.cpp -- continuous-batching walk server of liblabs.so.
//
// A scheduler thread owns a device memory pool.  Requests (one walk job of
// any L each) wait in a FIFO host queue; the head is admitted as soon as its
// footprint fits a free range of the pool.  Each launch of the persistent
// batch kernel runs every admitted request's unfinished walks, oldest request
// first; each walk's progress and visited table stay in the pool between
// launches.  By default a launch runs until its walks finish or until the
// scheduler asks it to stop (a host flag the kernel polls every 64 moves)
// because a queued request can be admitted or a running one has finished;
// the walks then save their state and the next launch, with the newcomers,
// resumes them.  With chunk_steps set, a launch advances every request by at
// most chunk_steps moves instead.  Completed requests are copied to host
// memory and their pool range is freed immediately.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "labs.h"
#include "labs_internal.h"

namespace {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

uint64_t al(uint64_t x) { return (x + 255) & ~(uint64_t)255; }

// First-fit allocator over [0, size) in 256-byte granules.
class RangeAlloc {
 public:
  void reset(uint64_t size) {
    free_.clear();
    if (size) free_[0] = size;
    used_ = peak_ = 0;
  }
  bool alloc(uint64_t bytes, uint64_t *off) {
    bytes = al(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const uint64_t rest = it->second - bytes;
        const uint64_t start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += bytes;
        peak_ = std::max(peak_, used_);
        return true;
      }
    }
    return false;
  }
  void release(uint64_t off, uint64_t bytes) {
    bytes = al(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  bool fits(uint64_t bytes) const {
    bytes = al(bytes);
    for (const auto &kv : free_)
      if (kv.second >= bytes) return true;
    return false;
  }
  uint64_t used() const { return used_; }
  uint64_t peak() const { return peak_; }

 private:
  std::map<uint64_t, uint64_t> free_;
  uint64_t used_ = 0, peak_ = 0;
};

enum { ST_PENDING = 0, ST_ACTIVE = 1, ST_DONE = 2 };

struct Request {
  uint64_t id;
  int32_t L;
  int64_t n_walks, walk_len;
  uint64_t seed;
  std::vector<uint64_t> starts;   // host copy, empty = seeded
  int32_t lanes;
  uint32_t n_buckets;
  uint64_t table_bytes;
  int W;
  // pool range and the buffers inside it
  uint64_t off = 0, bytes = 0;
  uint64_t o_tables = 0, o_state = 0, o_wstat = 0, o_starts = 0, o_seq = 0, o_E = 0, o_steps = 0,
           o_dig = 0;
  int64_t progress = 0;           // chunked launches: moves every still-moving walk has made
  bool launched = false;
  std::vector<uint8_t> walk_done; // walks known finished (host view)
  int64_t n_done = 0;
  bool upload = false;
  int status = ST_PENDING;
  int64_t t_submit = 0, t_admit = 0, t_done = 0;
  std::vector<uint64_t> h_seq, h_dig;
  std::vector<int32_t> h_E;
  std::vector<int64_t> h_steps;
};

constexpr int kMaxItems = 1 << 17;
// Control region: queue heads (one per kernel class, 64 bytes apart), then
// the work list and the instance table of the current launch.
constexpr uint64_t kCtlHead = 512;
constexpr int kMaxInst = 8192;
// Pinned host words the kernel reads and writes: the stop flag, then one
// completion word per work item of the current launch.
constexpr int kHostFlagWords = 64;

}  // namespace

struct labs_server {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t kstream = nullptr;    // the launches (default priority)
  bool full = false;                // whole-space requests (else skew-symmetric)
  uint8_t *pool = nullptr;          // control region, then request ranges
  uint64_t pool_bytes = 0;
  uint64_t ctl_bytes = 0;           // control region size
  int32_t max_pending = 4096;
  int32_t lanes = 0;
  int64_t chunk = 0;                // moves per launch; 0: run until done or asked to stop
  uint32_t *host_words = nullptr;   // pinned: stop flag, then item completion words
  uint32_t *dev_words = nullptr;    // the same memory as the kernel addresses it
  double load_factor = 0.5;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  hipError_t dev_err = hipSuccess;  // first device error; the server stops on it
  std::thread worker;
  std::deque<Request *> pending;
  std::vector<Request *> active;
  std::unordered_map<uint64_t, Request *> all;
  uint64_t next_id = 1;
  RangeAlloc ranges;
  labs_serve_counters st{};
};

namespace {

uint64_t footprint(Request &q) {
  uint64_t o = 0;
  q.o_tables = o; o += al((uint64_t)q.n_walks * q.table_bytes);
  q.o_state = o; o += al((uint64_t)q.n_walks * sizeof(lsaw::WalkState));
  q.o_wstat = o; o += al((uint64_t)q.n_walks);
  q.o_starts = o; o += q.starts.empty() ? 0 : al((uint64_t)q.n_walks * q.W * 8);
  q.o_seq = o; o += al((uint64_t)q.n_walks * q.W * 8);
  q.o_E = o; o += al((uint64_t)q.n_walks * 4);
  q.o_steps = o; o += al((uint64_t)q.n_walks * 8);
  q.o_dig = o; o += al((uint64_t)q.n_walks * 8);
  return o;
}

int64_t items_of(const Request &q, int lanes) {
  const int per = lsaw::kBlock / lanes;
  return (q.n_walks + per - 1) / per;
}

hipError_t finish(labs_server *s, Request *q) {
  q->h_seq.resize((size_t)q->n_walks * q->W);
  q->h_E.resize((size_t)q->n_walks);
  q->h_steps.resize((size_t)q->n_walks);
  q->h_dig.resize((size_t)q->n_walks);
  uint8_t *b = s->pool + s->ctl_bytes + q->off;
  hipError_t e = hipMemcpyAsync(q->h_seq.data(), b + q->o_seq, q->h_seq.size() * 8, hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(q->h_E.data(), b + q->o_E, q->h_E.size() * 4, hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(q->h_steps.data(), b + q->o_steps, q->h_steps.size() * 8, hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(q->h_dig.data(), b + q->o_dig, q->h_dig.size() * 8, hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  return e;
}

// Batch kernel (class group) that runs length L on this server.
int kernel_variant(const labs_server *s, int L) {
  return s->full ? lsaw::full_batch_variant(lsaw::full_lag_words_for(L))
                 : lsaw::batch_variant(lsaw::lag_words_for(L));
}

// Groups of `per` walks of q that still have an unfinished walk.
int64_t groups_left(const Request &q, int per) {
  int64_t n = 0;
  for (int64_t w = 0; w < q.n_walks; w += per) {
    const int64_t e = std::min<int64_t>(w + per, q.n_walks);
    for (int64_t x = w; x < e; ++x)
      if (!q.walk_done[(size_t)x]) {
        ++n;
        break;
      }
  }
  return n;
}

void run_worker(labs_server *s) {
  (void)hipSetDevice(s->device);
  std::vector<lsaw::BatchInstanceDev> inst;
  std::vector<lsaw::BatchItemDev> items;
  std::vector<int64_t> budget;
  volatile uint32_t *stop_flag = s->host_words;
  volatile uint32_t *item_done = s->host_words + kHostFlagWords;
  const bool preemptive = s->chunk == 0;
  for (;;) {
    std::vector<Request *> run;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      int64_t n_items = 0;
      for (Request *q : s->active) n_items += items_of(*q, 8);
      // first come, first served: the head waits until its footprint fits
      while (!s->pending.empty() && !s->stop) {
        Request *q = s->pending.front();
        if ((int64_t)s->active.size() + 1 > kMaxInst || n_items + items_of(*q, 8) > kMaxItems) break;
        uint64_t off = 0;
        if (!s->ranges.alloc(q->bytes, &off)) break;
        q->off = off;
        q->status = ST_ACTIVE;
        q->t_admit = now_ns();
        q->upload = !q->starts.empty();
        q->walk_done.assign((size_t)q->n_walks, 0);
        s->pending.pop_front();
        s->active.push_back(q);
        n_items += items_of(*q, 8);
        s->st.admitted++;
      }
      s->st.pool_used = s->ranges.used();
      s->st.pool_peak = s->ranges.peak();
      if (s->stop) break;
      if (s->active.empty()) {
        s->cv_work.wait(lk, [&] { return s->stop || !s->pending.empty(); });
        continue;
      }
      run = s->active;
    }
    // one launch over every admitted request
    inst.clear();
    items.clear();
    budget.clear();
    // One persistent grid per launch, on the kernel of the largest class
    // present (a shorter length runs exactly on a longer class's kernel).
    // Grids of several classes on separate streams would run concurrently
    // only if their streams sat on different hardware queues, which the
    // runtime does not promise; a grid queued behind another starves its
    // requests until the other ends.
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, s->device);
    int variant = 0;
    for (Request *q : run) variant = std::max(variant, kernel_variant(s, q->L));
    int per_cu = 1;
    if (s->full) (void)lsaw::full_batch_blocks_per_cu(variant, &per_cu, true);
    else (void)lsaw::batch_blocks_per_cu(variant, &per_cu, true);
    const int64_t slots = (int64_t)std::max(per_cu, 1) * cus;
    int64_t items4 = 0;
    for (Request *q : run) items4 += groups_left(*q, lsaw::kBlock / 4);
    // Lanes per walk for this launch (walk state and tables do not depend on
    // it): a request's own choice if it has one, else 4 or 8 (whole-space
    // walks: always 4).  Eight lanes cost about 20% more per walk step than
    // four (the per-move work is shared by half as many candidates per
    // lane), so they pay only where four leave resident workgroups idle.
    // Chunked launches run every item to the chunk's end, so what counts
    // there is how well the items fill whole rounds of workgroups; launches
    // that are stopped early keep every workgroup busy once the items fill
    // the device, and take eight lanes while four-lane items would fill less
    // than two thirds of the resident workgroups (measured on a mixed-L
    // stream: at 0.9x capacity 4-6 % more served throughput and a 17 % lower
    // p99 than a five-sixths threshold, and no loss when saturated).
    int lanes_auto = 4;
    if (!s->full) {
      if (preemptive) {
        lanes_auto = 3 * items4 < 2 * slots ? 8 : 4;
      } else {
        auto fill = [&](int64_t n) {
          const int64_t rounds = (n + slots - 1) / slots;
          return rounds > 0 ? (double)n / (double)(rounds * slots) : 0.0;
        };
        lanes_auto = 0.8 * fill(2 * items4) > fill(items4) ? 8 : 4;
      }
    }
    hipError_t up_err = hipSuccess;           // first failing upload or clear, if any
    for (size_t k = 0; k < run.size(); ++k) {
      Request *q = run[k];
      uint8_t *b = s->pool + s->ctl_bytes + q->off;
      if (q->upload) {
        if (up_err == hipSuccess)
          up_err = hipMemcpyAsync(b + q->o_starts, q->starts.data(), q->starts.size() * 8,
                                  hipMemcpyHostToDevice, s->stream);
        q->upload = false;
      }
      if (!q->launched && up_err == hipSuccess)   // every walk starts "not started"
        up_err = hipMemsetAsync(b + q->o_wstat, 0, (size_t)q->n_walks, s->stream);
      const int64_t take = preemptive ? q->walk_len : std::min(s->chunk, q->walk_len - q->progress);
      budget.push_back(take);
      lsaw::BatchInstanceDev d{};
      d.starts = q->starts.empty() ? nullptr : reinterpret_cast<const uint64_t *>(b + q->o_starts);
      d.seed = q->seed;
      d.walk_len = q->walk_len;
      d.best_seq = reinterpret_cast<uint64_t *>(b + q->o_seq);
      d.best_E = reinterpret_cast<int32_t *>(b + q->o_E);
      d.steps_done = reinterpret_cast<int64_t *>(b + q->o_steps);
      d.digest = reinterpret_cast<uint64_t *>(b + q->o_dig);
      d.trace_j = nullptr;
      d.trace_E = nullptr;
      d.n_trace = 0;
      d.table_bytes = q->table_bytes;
      d.n_buckets = q->n_buckets;
      d.L = q->L;
      d.tables = b + q->o_tables;
      d.state = reinterpret_cast<lsaw::WalkState *>(b + q->o_state);
      d.wstat = b + q->o_wstat;
      d.step_end = preemptive ? q->walk_len : q->progress + take;
      inst.push_back(d);
      const int lanes = q->lanes ? q->lanes : lanes_auto;
      const int per = lsaw::kBlock / lanes;
      for (int64_t w = 0; w < q->n_walks; w += per) {
        const int64_t n = std::min<int64_t>(per, q->n_walks - w);
        bool left = false;
        for (int64_t x = w; x < w + n && !left; ++x) left = !q->walk_done[(size_t)x];
        if (!left) continue;                  // every walk of the group has finished
        lsaw::BatchItemDev it{};
        it.inst = (int32_t)k;
        it.code = ((s->full ? lsaw::full_lag_words_for(q->L) : lsaw::lag_words_for(q->L)) << 4) | lanes;
        it.n_walks = (int32_t)n;
        it.walk_begin = w;
        items.push_back(it);
      }
    }
    // In chunked launches longest items first (cost grows with L, so the
    // persistent grid ends on short items), else oldest request first
    // (launches are cut short, so no grid tail to shape).
    std::stable_sort(items.begin(), items.end(), [&](const lsaw::BatchItemDev &x, const lsaw::BatchItemDev &y) {
      return preemptive ? x.inst < y.inst : inst[x.inst].L > inst[y.inst].L;
    });
    uint8_t *ctl = s->pool;
    const uint64_t items_off = kCtlHead;
    const uint64_t inst_off = al(items_off + (uint64_t)kMaxItems * sizeof(lsaw::BatchItemDev));
    lsaw::BatchLaunch bl;
    bl.items = reinterpret_cast<const lsaw::BatchItemDev *>(ctl + items_off);
    bl.n_items = (int64_t)items.size();
    bl.inst = reinterpret_cast<const lsaw::BatchInstanceDev *>(ctl + inst_off);
    bl.counter = reinterpret_cast<uint32_t *>(ctl);
    bl.arena = nullptr;                       // every instance brings its own tables
    bl.arena_bytes = 0;
    bl.preempt = preemptive ? s->dev_words : nullptr;
    bl.item_done = s->dev_words + kHostFlagWords;
    // No kernel runs now: the flag and the completion words can be reset.
    *stop_flag = 0u;
    for (size_t i = 0; i < items.size(); ++i) item_done[i] = 0u;
    const int64_t t0 = now_ns();
    hipError_t e = up_err;
    if (e == hipSuccess)
      e = hipMemcpyAsync(ctl + items_off, items.data(), items.size() * sizeof(lsaw::BatchItemDev),
                         hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(ctl + inst_off, inst.data(), inst.size() * sizeof(lsaw::BatchInstanceDev),
                         hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);   // work lists in place
    if (e == hipSuccess && !items.empty()) {
      const int grid = (int)std::min<int64_t>((int64_t)items.size(), slots);
      e = lsaw::launch_batch_reset(bl.counter, s->kstream);
      if (e == hipSuccess)
        e = s->full ? lsaw::launch_full_batch(bl, variant, grid, s->kstream, true)
                    : lsaw::launch_batch(bl, variant, grid, s->kstream, true);
    }
    if (preemptive && e == hipSuccess) {
      // Let the launch run until its walks finish, or ask it to stop (it then
      // ends within about 64 moves per walk) once a queued request can be
      // admitted, a running request has finished (so that it is delivered and
      // its memory freed now), or the server shuts down.
      bool asked = false;
      int64_t t_check = 0;
      std::vector<int64_t> left(run.size(), 0);
      for (;;) {
        const hipError_t qe = hipStreamQuery(s->kstream);
        if (qe != hipErrorNotReady) {
          if (qe != hipSuccess) e = qe;
          break;
        }
        if (!asked) {
          bool want = false;
          const int64_t t = now_ns();
          if (t - t_check > 2000000) {            // scan the completion words every 2 ms
            t_check = t;
            std::fill(left.begin(), left.end(), 0);
            for (size_t i = 0; i < items.size(); ++i)
              if (!item_done[i]) left[(size_t)items[i].inst]++;
            for (size_t k = 0; k < run.size() && !want; ++k) want = left[k] == 0;
          }
          std::unique_lock<std::mutex> lk(s->mu);
          want = want || s->stop || (!s->pending.empty() && s->ranges.fits(s->pending.front()->bytes));
          if (want) {
            *stop_flag = 1u;
            asked = true;
          } else {
            s->cv_work.wait_for(lk, std::chrono::microseconds(200));
          }
        }
        if (asked) std::this_thread::sleep_for(std::chrono::microseconds(100));
      }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s->kstream);
    const int64_t t1 = now_ns();
    // Items that ended with every walk finished, from the completion words.
    for (size_t i = 0; i < items.size() && e == hipSuccess; ++i) {
      if (!item_done[i]) continue;
      Request *q = run[(size_t)items[i].inst];
      for (int64_t x = items[i].walk_begin; x < items[i].walk_begin + items[i].n_walks; ++x)
        if (!q->walk_done[(size_t)x]) {
          q->walk_done[(size_t)x] = 1;
          q->n_done++;
        }
    }
    std::vector<Request *> done;
    for (size_t k = 0; k < run.size() && e == hipSuccess; ++k) {
      Request *q = run[k];
      q->launched = true;
      if (!preemptive) q->progress += budget[k];
      if (q->n_done == q->n_walks) {
        e = finish(s, q);
        done.push_back(q);
      }
    }
    if (e != hipSuccess) {
      // The device state of every admitted request is unknown now: stop, and
      // let poll / wait report the error for every unfinished request.
      {
        std::lock_guard<std::mutex> lk(s->mu);
        s->dev_err = e;
        s->stop = true;
      }
      s->cv_done.notify_all();
      break;
    }
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->st.launches++;
      s->st.busy_ns += t1 - t0;
      const int64_t tdone = now_ns();
      for (Request *q : done) {
        q->status = ST_DONE;
        q->t_done = tdone;
        int64_t tot = 0;
        for (int64_t v : q->h_steps) tot += v;
        s->st.walk_steps += tot;
        s->st.completed++;
        s->ranges.release(q->off, q->bytes);
        s->active.erase(std::find(s->active.begin(), s->active.end(), q));
      }
      s->st.pool_used = s->ranges.used();
    }
    if (!done.empty()) s->cv_done.notify_all();
  }
}

int32_t copy_result(Request *q, labs_serve_result *res) {
  if (!res) return LABS_OK;
  if (res->best_seq) memcpy(res->best_seq, q->h_seq.data(), q->h_seq.size() * 8);
  if (res->best_E) memcpy(res->best_E, q->h_E.data(), q->h_E.size() * 4);
  if (res->steps_done) memcpy(res->steps_done, q->h_steps.data(), q->h_steps.size() * 8);
  if (res->digest) memcpy(res->digest, q->h_dig.data(), q->h_dig.size() * 8);
  res->t_submit_ns = q->t_submit;
  res->t_admit_ns = q->t_admit;
  res->t_done_ns = q->t_done;
  int64_t tot = 0;
  for (int64_t v : q->h_steps) tot += v;
  res->total_steps = tot;
  return LABS_OK;
}

}  // namespace

extern "C" {

int32_t labs_serve_create(const labs_serve_cfg *cfg, labs_server **server) {
  if (!server) return lsaw::set_error(LABS_EINVAL, "NULL server");
  *server = nullptr;
  labs_serve_cfg c{};
  if (cfg) c = *cfg;
  if (c.max_pending < 0 || c.chunk_steps < 0) return lsaw::set_error(LABS_EINVAL, "negative configuration value");
  if (c.lanes_per_walk != 0 && c.lanes_per_walk != 2 && c.lanes_per_walk != 4 && c.lanes_per_walk != 8)
    return lsaw::set_error(LABS_EINVAL, "lanes_per_walk=%d: use 0, 2, 4 or 8", c.lanes_per_walk);
  if (c.load_factor != 0.0 && !(c.load_factor > 0.0 && c.load_factor <= 0.9))
    return lsaw::set_error(LABS_EINVAL, "load_factor=%g: use 0 or a value in (0, 0.9]", c.load_factor);
  if (c.whole_space != 0 && c.whole_space != 1)
    return lsaw::set_error(LABS_EINVAL, "whole_space=%d: use 0 or 1", c.whole_space);
  if (c.whole_space && c.lanes_per_walk != 0 && c.lanes_per_walk != lsaw::full_lanes_per_walk())
    return lsaw::set_error(LABS_EINVAL, "lanes_per_walk=%d: whole-space walks use 0 or %d", c.lanes_per_walk,
                           lsaw::full_lanes_per_walk());
  labs_server *s = new labs_server();
  s->full = c.whole_space != 0;
  s->max_pending = c.max_pending ? c.max_pending : 4096;
  s->lanes = c.lanes_per_walk;
  s->chunk = c.chunk_steps;
  s->load_factor = c.load_factor != 0.0 ? c.load_factor : 0.0;
  hipError_t e = hipGetDevice(&s->device);
  size_t free_b = 0, total_b = 0;
  if (e == hipSuccess) e = hipMemGetInfo(&free_b, &total_b);
  s->ctl_bytes = al(kCtlHead + (uint64_t)kMaxItems * sizeof(lsaw::BatchItemDev)) +
                 al((uint64_t)kMaxInst * sizeof(lsaw::BatchInstanceDev));
  uint64_t want = c.pool_bytes ? c.pool_bytes : (uint64_t)(free_b / 2);
  want = al(want);
  if (e == hipSuccess && want <= s->ctl_bytes) e = hipErrorInvalidValue;
  if (e == hipSuccess) e = hipMalloc(&s->pool, want);
  // Coherent pinned words: the scheduler raises the stop flag while a launch
  // runs and reads the kernel's item completion words.
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void **>(&s->host_words),
                      (size_t)(kHostFlagWords + kMaxItems) * sizeof(uint32_t),
                      hipHostMallocMapped | hipHostMallocCoherent);
  if (e == hipSuccess)
    e = hipHostGetDevicePointer(reinterpret_cast<void **>(&s->dev_words), s->host_words, 0);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->kstream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    if (s->stream) (void)hipStreamDestroy(s->stream);
    if (s->kstream) (void)hipStreamDestroy(s->kstream);
    if (s->pool) (void)hipFree(s->pool);
    if (s->host_words) (void)hipHostFree(s->host_words);
    delete s;
    return lsaw::set_error(e == hipErrorOutOfMemory ? LABS_ENOMEM : LABS_EDEVICE, "serve create: %s",
                           hipGetErrorString(e));
  }
  s->pool_bytes = want;
  s->ranges.reset(want - s->ctl_bytes);
  s->st.pool_bytes = want - s->ctl_bytes;
  s->worker = std::thread(run_worker, s);
  *server = s;
  return lsaw::clear_error();
}

int32_t labs_serve_destroy(labs_server *s) {
  if (!s) return lsaw::clear_error();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (auto &kv : s->all) delete kv.second;
  if (s->stream) (void)hipStreamDestroy(s->stream);
  if (s->kstream) (void)hipStreamDestroy(s->kstream);
  if (s->pool) (void)hipFree(s->pool);
  if (s->host_words) (void)hipHostFree(s->host_words);
  delete s;
  return lsaw::clear_error();
}

int32_t labs_serve_submit(labs_server *s, int32_t L, int64_t n_walks, int64_t walk_len, uint64_t seed,
                          const uint64_t *starts, uint64_t *req_id) {
  if (!s || !req_id) return lsaw::set_error(LABS_EINVAL, "NULL server or req_id");
  if (n_walks <= 0) return lsaw::set_error(LABS_EINVAL, "n_walks=%lld must be > 0", (long long)n_walks);
  const int32_t lanes = s->full ? lsaw::full_lanes_per_walk() : s->lanes;   // 0: chosen per launch
  if (s->full ? !(L >= 3 && L <= lsaw::kFullLMax) : !(L >= 3 && L <= lsaw::kLMax && (L & 1)))
    return lsaw::set_error(LABS_EINVAL, s->full ? "L=%d: need 3 <= L <= %d" : "L=%d: need odd L with 3 <= L <= %d",
                           L, s->full ? lsaw::kFullLMax : lsaw::kLMax);
  double lf = s->load_factor;
  if (lf == 0.0) {
    int32_t tl = 4;
    double tf = 0.5;
    if (!s->full) lsaw::tuned_plan(L, &tl, &tf);
    lf = tf;
  }
  uint32_t nb = 0;
  uint64_t tb = 0;
  if (walk_len < 0) return lsaw::set_error(LABS_EINVAL, "walk_len must be >= 0");
  if (!lsaw::table_geometry(L, walk_len, lf, &nb, &tb, s->full)) return LABS_EINVAL;
  Request *q = new Request();
  q->L = L;
  q->n_walks = n_walks;
  q->walk_len = walk_len;
  q->seed = seed;
  q->lanes = lanes;
  q->n_buckets = nb;
  q->table_bytes = tb;
  q->W = s->full ? lsaw::full_key_words_for(L) : lsaw::key_words_for(L);
  if (starts) {
    q->starts.assign(starts, starts + (size_t)n_walks * q->W);
    const int bits = s->full ? L : lsaw::free_bits(L);   // key bits
    const int top = bits - 64 * (q->W - 1);
    for (int64_t w = 0; w < n_walks; ++w)
      if (top < 64 && (q->starts[(size_t)w * q->W + q->W - 1] >> top) != 0) {
        delete q;
        return lsaw::set_error(LABS_EINVAL, "start %lld has bits above the %d key bits", (long long)w, bits);
      }
  }
  q->bytes = footprint(*q);
  if (q->bytes > s->pool_bytes - s->ctl_bytes || items_of(*q, 8) > kMaxItems) {
    const unsigned long long need = q->bytes;
    delete q;
    return lsaw::set_error(LABS_EINVAL, "request footprint %llu bytes exceeds the pool", need);
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
      delete q;
      return lsaw::set_error(LABS_EDEVICE, "server stopped");
    }
    if ((int32_t)s->pending.size() >= s->max_pending) {
      delete q;
      return lsaw::set_error(LABS_EBUSY, "request queue full (%d pending)", s->max_pending);
    }
    q->id = s->next_id++;
    q->t_submit = now_ns();
    s->pending.push_back(q);
    s->all[q->id] = q;
    s->st.submitted++;
    *req_id = q->id;
  }
  s->cv_work.notify_one();
  return lsaw::clear_error();
}

int32_t labs_serve_poll(labs_server *s, uint64_t req_id, labs_serve_result *res) {
  if (!s) return lsaw::set_error(LABS_EINVAL, "NULL server");
  Request *q = nullptr;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(req_id);
    if (it == s->all.end()) return lsaw::set_error(LABS_ENOTFOUND, "unknown request %llu", (unsigned long long)req_id);
    if (it->second->status != ST_DONE) {
      if (s->dev_err != hipSuccess)
        return lsaw::set_error(LABS_EDEVICE, "server stopped on a device error: %s", hipGetErrorString(s->dev_err));
      return LABS_PENDING;
    }
    q = it->second;
    s->all.erase(it);
  }
  copy_result(q, res);
  delete q;
  return lsaw::clear_error();
}

int32_t labs_serve_wait(labs_server *s, uint64_t req_id, int64_t timeout_ns, labs_serve_result *res) {
  if (!s) return lsaw::set_error(LABS_EINVAL, "NULL server");
  {
    std::unique_lock<std::mutex> lk(s->mu);
    auto done = [&] {
      auto it = s->all.find(req_id);
      return it == s->all.end() || it->second->status == ST_DONE || s->stop;
    };
    if (timeout_ns < 0) s->cv_done.wait(lk, done);
    else s->cv_done.wait_for(lk, std::chrono::nanoseconds(timeout_ns), done);
  }
  return labs_serve_poll(s, req_id, res);
}

int32_t labs_serve_stats(labs_server *s, labs_serve_counters *out) {
  if (!s || !out) return lsaw::set_error(LABS_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->st;
  out->pending = (int64_t)s->pending.size();
  out->active = (int64_t)s->active.size();
  return lsaw::clear_error();
}

}  // extern "C"
