// labs_api.cpp -- host side of liblabs.so: argument validation, workspace
// sizing, launch planning and the packed-key helpers of include/labs.h.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>
#include <stdarg.h>
#include <algorithm>
#include <string>

#include "labs.h"
#include "labs_internal.h"

namespace {

thread_local std::string g_err;

int32_t fail(int32_t code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int32_t ok() {
  g_err.clear();
  return LABS_OK;
}

bool valid_skew_L(int32_t L) { return L >= 3 && L <= lsaw::kLMax && (L & 1) == 1; }

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

struct Plan {
  int G;                 // lanes per walk
  double alpha;          // table load factor bound
  uint32_t n_buckets;    // buckets per walk
  uint64_t table_bytes;  // bytes per walk
  int64_t max_conc;      // user bound on resident walks (0 = none)
};

// Plan fields from the caller's labs_plan and the visited-table size for
// walk_len moves with entries of entry_bytes.
int32_t plan_tables(int entry_bytes, int64_t walk_len, const labs_plan *p, Plan &out) {
  if (walk_len < 0) return fail(LABS_EINVAL, "walk_len=%lld must be >= 0", (long long)walk_len);
  if (walk_len > (int64_t)1 << 31) return fail(LABS_EINVAL, "walk_len=%lld exceeds 2^31", (long long)walk_len);
  out.G = 0;
  out.alpha = 0.5;
  out.max_conc = 0;
  if (p) {
    if (p->lanes_per_walk != 0 && p->lanes_per_walk != 1 && p->lanes_per_walk != 2 &&
        p->lanes_per_walk != 4 && p->lanes_per_walk != 8)
      return fail(LABS_EINVAL, "lanes_per_walk=%d: use 0, 1, 2, 4 or 8", p->lanes_per_walk);
    if (p->load_factor != 0.0 && !(p->load_factor > 0.0 && p->load_factor <= 0.9))
      return fail(LABS_EINVAL, "load_factor=%g: use 0 or a value in (0, 0.9]", p->load_factor);
    if (p->max_concurrent < 0) return fail(LABS_EINVAL, "max_concurrent must be >= 0");
    out.G = p->lanes_per_walk;
    if (p->load_factor != 0.0) out.alpha = p->load_factor;
    out.max_conc = p->max_concurrent;
  }
  const int epb = lsaw::kBucketBytes / entry_bytes;
  const double keys = (double)walk_len + 1.0;
  double nb = keys / (epb * out.alpha);
  uint64_t n_buckets = (uint64_t)nb;
  if ((double)n_buckets < nb) ++n_buckets;
  if (n_buckets < 1) n_buckets = 1;
  // The table must always keep a free entry so that every probe terminates.
  while (n_buckets * (uint64_t)epb <= (uint64_t)walk_len + 1) ++n_buckets;
  if (n_buckets >= ((uint64_t)1 << 32)) return fail(LABS_EINVAL, "visited table too large");
  out.n_buckets = (uint32_t)n_buckets;
  out.table_bytes = n_buckets * (uint64_t)lsaw::kBucketBytes;
  return LABS_OK;
}

int32_t make_plan(int32_t L, int64_t walk_len, const labs_plan *p, Plan &out) {
  if (!valid_skew_L(L)) return fail(LABS_EINVAL, "L=%d: need odd L with 3 <= L <= %d", L, lsaw::kLMax);
  return plan_tables(lsaw::entry_bytes_for(L), walk_len, p, out);
}

bool valid_full_L(int32_t L) { return L >= 3 && L <= lsaw::kFullLMax; }

// Whole-space walks run four lanes per walk.
int32_t make_full_plan(int32_t L, int64_t walk_len, const labs_plan *p, Plan &out) {
  if (!valid_full_L(L)) return fail(LABS_EINVAL, "L=%d: need 3 <= L <= %d", L, lsaw::kFullLMax);
  const int32_t rc = plan_tables(lsaw::full_entry_bytes_for(L), walk_len, p, out);
  if (rc != LABS_OK) return rc;
  const int G = lsaw::full_lanes_per_walk();
  if (out.G != 0 && out.G != G)
    return fail(LABS_EINVAL, "lanes_per_walk=%d: whole-space walks use 0 or %d", out.G, G);
  out.G = G;
  return LABS_OK;
}

// Lanes per walk when the caller leaves it to the library: enough lanes to
// give every SIMD of the 256-CU chip about two resident wavefronts.
int auto_lanes(int64_t concurrent) {
  const int64_t target = 256LL * 4 * 64 * 2;
  int G = 1;
  while (G < 8 && concurrent * G < target) G *= 2;
  return G;
}

}  // namespace

extern "C" {

const char *labs_last_error(void) { return g_err.c_str(); }

int32_t labs_l_max(void) { return lsaw::kLMax; }

int32_t labs_key_words(int32_t L) { return valid_skew_L(L) ? lsaw::key_words_for(L) : 0; }

int32_t labs_energy(const int8_t *seqs, int32_t L, int64_t n, int32_t *E_out, void *stream) {
  if (L < 1 || L > lsaw::kEnergyLMax) return fail(LABS_EINVAL, "L=%d: need 1 <= L <= %d", L, lsaw::kEnergyLMax);
  if (n < 0) return fail(LABS_EINVAL, "n=%lld must be >= 0", (long long)n);
  if (n > 0 && (!seqs || !E_out)) return fail(LABS_EINVAL, "NULL buffer");
  hipError_t e = lsaw::launch_energy(seqs, L, n, E_out, as_stream(stream));
  if (e != hipSuccess) return fail(LABS_EDEVICE, "energy launch: %s", hipGetErrorString(e));
  return ok();
}

int32_t labs_pack_skew(const int8_t *x, int32_t L, int64_t n, uint64_t *out) {
  if (!valid_skew_L(L)) return fail(LABS_EINVAL, "L=%d: need odd L with 3 <= L <= %d", L, lsaw::kLMax);
  if (n < 0) return fail(LABS_EINVAL, "n must be >= 0");
  if (n > 0 && (!x || !out)) return fail(LABS_EINVAL, "NULL buffer");
  const int D = lsaw::free_bits(L), W = lsaw::key_words_for(L);
  for (int64_t s = 0; s < n; ++s) {
    for (int w = 0; w < W; ++w) out[s * W + w] = 0;
    for (int j = 0; j < D; ++j) {
      const int8_t v = x[s * D + j];
      if (v != 1 && v != -1) return fail(LABS_EINVAL, "element %lld,%d is %d, not +-1", (long long)s, j, (int)v);
      if (v < 0) out[s * W + j / 64] |= (uint64_t)1 << (j % 64);
    }
  }
  return ok();
}

int32_t labs_unpack_skew(const uint64_t *keys, int32_t L, int64_t n, int8_t *x) {
  if (!valid_skew_L(L)) return fail(LABS_EINVAL, "L=%d: need odd L with 3 <= L <= %d", L, lsaw::kLMax);
  if (n < 0) return fail(LABS_EINVAL, "n must be >= 0");
  if (n > 0 && (!keys || !x)) return fail(LABS_EINVAL, "NULL buffer");
  const int D = lsaw::free_bits(L), W = lsaw::key_words_for(L);
  for (int64_t s = 0; s < n; ++s) {
    const int top = D - 64 * (W - 1);
    if (top < 64 && (keys[s * W + W - 1] >> top) != 0)
      return fail(LABS_EINVAL, "key %lld has bits above D=%d", (long long)s, D);
    for (int j = 0; j < D; ++j)
      x[s * D + j] = ((keys[s * W + j / 64] >> (j % 64)) & 1u) ? (int8_t)-1 : (int8_t)1;
  }
  return ok();
}

int32_t labs_expand_skew(const int8_t *x, int32_t L, int64_t n, int8_t *s) {
  if (!valid_skew_L(L)) return fail(LABS_EINVAL, "L=%d: need odd L with 3 <= L <= %d", L, lsaw::kLMax);
  if (n < 0) return fail(LABS_EINVAL, "n must be >= 0");
  if (n > 0 && (!x || !s)) return fail(LABS_EINVAL, "NULL buffer");
  const int D = lsaw::free_bits(L);
  for (int64_t q = 0; q < n; ++q) {
    const int8_t *xi = x + q * D;
    int8_t *so = s + q * L;
    for (int j = 0; j < D; ++j) {
      if (xi[j] != 1 && xi[j] != -1) return fail(LABS_EINVAL, "element %lld,%d is not +-1", (long long)q, j);
      so[j] = xi[j];
    }
    for (int i = 1; i <= D - 1; ++i) so[D + i - 1] = (i & 1) ? (int8_t)(-so[D - i - 1]) : so[D - i - 1];
  }
  return ok();
}

int32_t labs_starts(int32_t L, int64_t n_walks, uint64_t seed, uint64_t *out, void *stream) {
  if (!valid_skew_L(L)) return fail(LABS_EINVAL, "L=%d: need odd L with 3 <= L <= %d", L, lsaw::kLMax);
  if (n_walks < 0) return fail(LABS_EINVAL, "n_walks must be >= 0");
  if (n_walks > 0 && !out) return fail(LABS_EINVAL, "NULL buffer");
  hipError_t e = lsaw::launch_starts(L, n_walks, seed, out, as_stream(stream));
  if (e != hipSuccess) return fail(LABS_EDEVICE, "starts launch: %s", hipGetErrorString(e));
  return ok();
}

int32_t labs_walks_workspace_bytes(int32_t L, int64_t n_walks, int64_t walk_len,
                                   const labs_plan *plan, uint64_t *bytes) {
  if (!bytes) return fail(LABS_EINVAL, "NULL bytes");
  if (n_walks < 0) return fail(LABS_EINVAL, "n_walks must be >= 0");
  Plan p;
  int32_t rc = make_plan(L, walk_len, plan, p);
  if (rc != LABS_OK) return rc;
  int64_t conc = n_walks;
  if (p.max_conc > 0) conc = std::min(conc, p.max_conc);
  *bytes = (uint64_t)conc * p.table_bytes;
  return ok();
}

int32_t labs_walks_min_workspace_bytes(int32_t L, int64_t walk_len, const labs_plan *plan,
                                       uint64_t *bytes) {
  if (!bytes) return fail(LABS_EINVAL, "NULL bytes");
  Plan p;
  int32_t rc = make_plan(L, walk_len, plan, p);
  if (rc != LABS_OK) return rc;
  *bytes = p.table_bytes;
  return ok();
}

int32_t labs_walks(const uint64_t *starts, int32_t L, int64_t n_walks, int64_t walk_len,
                   uint64_t seed, const labs_walk_out *out, void *workspace, uint64_t ws_bytes,
                   const labs_plan *plan, void *stream) {
  Plan p;
  int32_t rc = make_plan(L, walk_len, plan, p);
  if (rc != LABS_OK) return rc;
  if (n_walks < 0) return fail(LABS_EINVAL, "n_walks=%lld must be >= 0", (long long)n_walks);
  if (!out) return fail(LABS_EINVAL, "NULL out");
  if (n_walks == 0) return ok();
  if (!out->best_seq || !out->best_E || !out->steps_done)
    return fail(LABS_EINVAL, "best_seq, best_E and steps_done are required");
  if (out->n_trace < 0 || out->n_trace > n_walks) return fail(LABS_EINVAL, "n_trace out of range");
  if (out->n_trace > 0 && (!out->trace_j || !out->trace_E))
    return fail(LABS_EINVAL, "trace buffers required when n_trace > 0");
  if (!workspace) return fail(LABS_EINVAL, "NULL workspace");
  if (ws_bytes < p.table_bytes)
    return fail(LABS_EINVAL, "workspace of %llu bytes is below the minimum %llu",
                (unsigned long long)ws_bytes, (unsigned long long)p.table_bytes);
  int64_t conc = (int64_t)std::min<uint64_t>((uint64_t)n_walks, ws_bytes / p.table_bytes);
  if (p.max_conc > 0) conc = std::min(conc, p.max_conc);
  const int G = p.G ? p.G : auto_lanes(conc);
  hipStream_t st = as_stream(stream);
  for (int64_t begin = 0; begin < n_walks; begin += conc) {
    const int64_t cnt = std::min(conc, n_walks - begin);
    lsaw::WalkLaunch w;
    w.starts = starts;
    w.seed = seed;
    w.L = L;
    w.walk_begin = begin;
    w.n_walks = cnt;
    w.walk_len = walk_len;
    w.best_seq = out->best_seq;
    w.best_E = out->best_E;
    w.steps_done = out->steps_done;
    w.digest = out->digest;
    w.trace_j = out->trace_j;
    w.trace_E = out->trace_E;
    w.n_trace = out->n_trace;
    w.cap_steps = out->cap_steps;
    w.tables = static_cast<uint8_t *>(workspace);
    w.table_bytes = p.table_bytes;
    w.n_buckets = p.n_buckets;
    w.lanes_per_walk = G;
    hipError_t e = lsaw::launch_walks(w, st);
    if (e != hipSuccess) return fail(LABS_EDEVICE, "walk launch: %s", hipGetErrorString(e));
  }
  return ok();
}

int32_t labs_full_l_max(void) { return lsaw::kFullLMax; }

int32_t labs_full_key_words(int32_t L) { return valid_full_L(L) ? lsaw::full_key_words_for(L) : 0; }

int32_t labs_full_walks_workspace_bytes(int32_t L, int64_t n_walks, int64_t walk_len,
                                        const labs_plan *plan, uint64_t *bytes) {
  if (!bytes) return fail(LABS_EINVAL, "NULL bytes");
  if (n_walks < 0) return fail(LABS_EINVAL, "n_walks must be >= 0");
  Plan p;
  int32_t rc = make_full_plan(L, walk_len, plan, p);
  if (rc != LABS_OK) return rc;
  int64_t conc = n_walks;
  if (p.max_conc > 0) conc = std::min(conc, p.max_conc);
  *bytes = (uint64_t)conc * p.table_bytes;
  return ok();
}

int32_t labs_full_walks(const uint64_t *starts, int32_t L, int64_t n_walks, int64_t walk_len,
                        uint64_t seed, const labs_walk_out *out, void *workspace, uint64_t ws_bytes,
                        const labs_plan *plan, void *stream) {
  Plan p;
  int32_t rc = make_full_plan(L, walk_len, plan, p);
  if (rc != LABS_OK) return rc;
  if (n_walks < 0) return fail(LABS_EINVAL, "n_walks=%lld must be >= 0", (long long)n_walks);
  if (!out) return fail(LABS_EINVAL, "NULL out");
  if (n_walks == 0) return ok();
  if (!out->best_seq || !out->best_E || !out->steps_done)
    return fail(LABS_EINVAL, "best_seq, best_E and steps_done are required");
  if (out->n_trace < 0 || out->n_trace > n_walks) return fail(LABS_EINVAL, "n_trace out of range");
  if (out->n_trace > 0 && (!out->trace_j || !out->trace_E))
    return fail(LABS_EINVAL, "trace buffers required when n_trace > 0");
  if (!workspace) return fail(LABS_EINVAL, "NULL workspace");
  if (ws_bytes < p.table_bytes)
    return fail(LABS_EINVAL, "workspace of %llu bytes is below the minimum %llu",
                (unsigned long long)ws_bytes, (unsigned long long)p.table_bytes);
  int64_t conc = (int64_t)std::min<uint64_t>((uint64_t)n_walks, ws_bytes / p.table_bytes);
  if (p.max_conc > 0) conc = std::min(conc, p.max_conc);
  hipStream_t st = as_stream(stream);
  for (int64_t begin = 0; begin < n_walks; begin += conc) {
    const int64_t cnt = std::min(conc, n_walks - begin);
    lsaw::WalkLaunch w;
    w.starts = starts;
    w.seed = seed;
    w.L = L;
    w.walk_begin = begin;
    w.n_walks = cnt;
    w.walk_len = walk_len;
    w.best_seq = out->best_seq;
    w.best_E = out->best_E;
    w.steps_done = out->steps_done;
    w.digest = out->digest;
    w.trace_j = out->trace_j;
    w.trace_E = out->trace_E;
    w.n_trace = out->n_trace;
    w.cap_steps = out->cap_steps;
    w.tables = static_cast<uint8_t *>(workspace);
    w.table_bytes = p.table_bytes;
    w.n_buckets = p.n_buckets;
    w.lanes_per_walk = p.G;
    hipError_t e = lsaw::launch_full_walks(w, st);
    if (e != hipSuccess) return fail(LABS_EDEVICE, "whole-space walk launch: %s", hipGetErrorString(e));
  }
  return ok();
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Mixed-length batches, their hipGraph form, and the per-L tuning table
// ---------------------------------------------------------------------------
#include <map>
#include <mutex>
#include <vector>

namespace {

struct Tuned {
  int32_t lanes;
  double load_factor;
};

std::mutex g_tune_mu;
std::map<int32_t, Tuned> g_tune;

// Built-in choice when L has no tuned entry: four lanes per walk (the fastest
// setting measured at L = 101 and L = 151 with tens of thousands of walks).
Tuned tuned_for(int32_t L) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(L);
  if (it != g_tune.end()) return it->second;
  return Tuned{4, 0.5};
}

constexpr int kMaxGroups = 8;          // more than the kernel classes (2..6)
constexpr uint64_t kQueueHeads = 512;  // queue heads at 64-byte spacing, then the work list

struct BatchGroup {
  int variant;              // batch kernel (lag-word class) of these items
  int64_t begin, count;     // their range in the item list
};

struct BatchPlan {
  bool full = false;                         // whole-space instances (labs_full_walks_batch)
  std::vector<lsaw::BatchInstanceDev> inst;
  std::vector<lsaw::BatchItemDev> items;
  std::vector<BatchGroup> groups;            // one persistent launch each, in order
  uint64_t arena_bytes;
  uint64_t items_off, inst_off, arena_off;   // byte offsets in the workspace
};

uint64_t align256(uint64_t x) { return (x + 255) & ~(uint64_t)255; }

int32_t plan_batch(const labs_instance *in, int32_t n_inst, BatchPlan &bp, bool full = false) {
  if (n_inst < 0) return fail(LABS_EINVAL, "n_inst must be >= 0");
  if (n_inst > 0 && !in) return fail(LABS_EINVAL, "NULL instance array");
  bp.full = full;
  bp.inst.clear();
  bp.items.clear();
  bp.groups.clear();
  bp.arena_bytes = 0;
  struct Ord { int variant, G, L, idx; };
  std::vector<Ord> order;
  for (int32_t i = 0; i < n_inst; ++i) {
    const labs_instance &x = in[i];
    labs_plan lp{x.lanes_per_walk, x.load_factor, 0};
    Plan p;
    if (full) {
      // whole space: four lanes per walk, load factor as given or 0.5
      int32_t rc = make_full_plan(x.L, x.walk_len, &lp, p);
      if (rc != LABS_OK) return fail(rc, "instance %d: %s", i, g_err.c_str());
      lp.lanes_per_walk = p.G;
    } else {
      const Tuned tu = tuned_for(x.L);
      if (lp.lanes_per_walk == 0) lp.lanes_per_walk = tu.lanes;
      if (lp.load_factor == 0.0) lp.load_factor = tu.load_factor;
      if (lp.lanes_per_walk != 2 && lp.lanes_per_walk != 4 && lp.lanes_per_walk != 8)
        return fail(LABS_EINVAL, "instance %d: lanes_per_walk %d (batches use 2, 4 or 8)", i,
                    lp.lanes_per_walk);
      int32_t rc = make_plan(x.L, x.walk_len, &lp, p);
      if (rc != LABS_OK) return fail(rc, "instance %d: %s", i, g_err.c_str());
    }
    if (x.n_walks < 0) return fail(LABS_EINVAL, "instance %d: n_walks < 0", i);
    if (x.n_walks > 0 && (!x.out.best_seq || !x.out.best_E || !x.out.steps_done))
      return fail(LABS_EINVAL, "instance %d: best_seq, best_E and steps_done are required", i);
    if (x.out.n_trace < 0 || x.out.n_trace > x.n_walks)
      return fail(LABS_EINVAL, "instance %d: n_trace out of range", i);
    if (x.out.n_trace > 0 && (!x.out.trace_j || !x.out.trace_E))
      return fail(LABS_EINVAL, "instance %d: trace buffers required", i);
    lsaw::BatchInstanceDev d{};
    d.starts = x.starts;
    d.seed = x.seed;
    d.walk_len = x.walk_len;
    d.best_seq = x.out.best_seq;
    d.best_E = x.out.best_E;
    d.cap_steps = x.out.cap_steps;
    d.steps_done = x.out.steps_done;
    d.digest = x.out.digest;
    d.trace_j = x.out.trace_j;
    d.trace_E = x.out.trace_E;
    d.n_trace = x.out.n_trace;
    d.table_bytes = p.table_bytes;
    d.n_buckets = p.n_buckets;
    d.L = x.L;
    d.tables = nullptr;
    d.state = nullptr;
    d.wstat = nullptr;
    d.step_end = x.walk_len;
    bp.inst.push_back(d);
    const int per_block = lsaw::kBlock / lp.lanes_per_walk;
    bp.arena_bytes = std::max(bp.arena_bytes, (uint64_t)per_block * p.table_bytes);
    const int variant = full ? lsaw::full_batch_variant(lsaw::full_lag_words_for(x.L))
                             : lsaw::batch_variant(lsaw::lag_words_for(x.L));
    order.push_back(Ord{variant, lp.lanes_per_walk, x.L, i});
  }
  // Classes whose kernels reach the same occupancy share one launch on the
  // largest class's kernel (a shorter length runs on a longer class's kernel
  // exactly): separate launches would only add tails.  (The whole-space
  // kernel groups are formed that way already.)
  if (!full) {
    int present[8] = {0};
    for (const Ord &o : order) present[o.variant] = 1;
    int merged[8] = {0, 0, 2, 3, 4, 5, 6, 6};
    int top = 0, top_occ = 0;
    for (int v = 6; v >= 2; --v) {
      if (!present[v]) continue;
      int occ = 0;
      if (lsaw::batch_blocks_per_cu(v, &occ) != hipSuccess) occ = 0;
      if (top && occ <= top_occ) {
        merged[v] = top;
      } else {
        top = v;
        top_occ = occ;
      }
    }
    for (Ord &o : order) o.variant = merged[o.variant];
  }
  // One launch per lag-word class (each at its own occupancy), largest class
  // first; inside a class the longest items first (cost grows with L), so a
  // persistent grid ends on short items and its tail stays short.
  std::stable_sort(order.begin(), order.end(), [](const Ord &a, const Ord &b) {
    if (a.variant != b.variant) return a.variant > b.variant;
    if (a.L != b.L) return a.L > b.L;
    return a.G < b.G;
  });
  for (const Ord &o : order) {
    const int per_block = lsaw::kBlock / o.G;
    const int64_t n = in[o.idx].n_walks;
    if (n > 0 && (bp.groups.empty() || bp.groups.back().variant != o.variant))
      bp.groups.push_back(BatchGroup{o.variant, (int64_t)bp.items.size(), 0});
    for (int64_t b = 0; b < n; b += per_block) {
      lsaw::BatchItemDev it{};
      it.inst = o.idx;
      it.code = ((full ? lsaw::full_lag_words_for(in[o.idx].L) : lsaw::lag_words_for(in[o.idx].L)) << 4) | o.G;
      it.n_walks = (int32_t)std::min<int64_t>(per_block, n - b);
      it.walk_begin = b;
      bp.items.push_back(it);
      bp.groups.back().count++;
    }
  }
  bp.items_off = kQueueHeads;
  bp.inst_off = align256(bp.items_off + bp.items.size() * sizeof(lsaw::BatchItemDev));
  bp.arena_off = align256(bp.inst_off + bp.inst.size() * sizeof(lsaw::BatchInstanceDev));
  return LABS_OK;
}

int32_t device_resident_blocks(int variant, bool full, int64_t *blocks) {
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = full ? lsaw::full_batch_blocks_per_cu(variant, &per_cu) : lsaw::batch_blocks_per_cu(variant, &per_cu);
  if (e != hipSuccess) return fail(LABS_EDEVICE, "device query: %s", hipGetErrorString(e));
  *blocks = (int64_t)std::max(1, per_cu) * (int64_t)cus;
  return LABS_OK;
}

// Persistent grids of the groups: resident workgroups of each kernel, at most
// one per item.  The groups run concurrently when the workspace holds a slice
// for every workgroup of every group, else one after another with each grid
// cut to the slices there are.
int32_t batch_grids(const BatchPlan &bp, uint64_t ws_bytes, std::vector<int> &grids, bool *concurrent) {
  grids.clear();
  if (ws_bytes < bp.arena_off + bp.arena_bytes)
    return fail(LABS_EINVAL, "workspace of %llu bytes is below the minimum %llu",
                (unsigned long long)ws_bytes, (unsigned long long)(bp.arena_off + bp.arena_bytes));
  const uint64_t fit = (ws_bytes - bp.arena_off) / std::max<uint64_t>(bp.arena_bytes, 1);
  uint64_t total = 0;
  for (const BatchGroup &grp : bp.groups) {
    int64_t resident = 0;
    int32_t rc = device_resident_blocks(grp.variant, bp.full, &resident);
    if (rc != LABS_OK) return rc;
    grids.push_back((int)std::min<int64_t>(grp.count, resident));
    total += (uint64_t)grids.back();
  }
  *concurrent = total <= fit;
  if (!*concurrent)
    for (int &g : grids) g = (int)std::min<uint64_t>((uint64_t)g, fit);
  return LABS_OK;
}

lsaw::BatchLaunch batch_launch(const BatchPlan &bp, uint8_t *ws, size_t k) {
  const BatchGroup &grp = bp.groups[k];
  lsaw::BatchLaunch b;
  b.items = reinterpret_cast<const lsaw::BatchItemDev *>(ws + bp.items_off) + grp.begin;
  b.n_items = grp.count;
  b.inst = reinterpret_cast<const lsaw::BatchInstanceDev *>(ws + bp.inst_off);
  b.counter = reinterpret_cast<uint32_t *>(ws + 64 * k);      // own queue head per group
  b.arena = ws + bp.arena_off;
  b.arena_bytes = bp.arena_bytes;
  b.preempt = nullptr;
  b.item_done = nullptr;
  return b;
}

// Library-owned side streams (default priority) and fork/join events of one
// device, created on first use.  Group 0 of a batch runs on the caller's
// stream and group k on side stream k; the groups hold disjoint instances,
// their own queue heads and disjoint ranges of arena slices.
struct SideStreams {
  hipStream_t s[kMaxGroups] = {nullptr};
  hipEvent_t fork = nullptr, join[kMaxGroups] = {nullptr};
};
std::mutex g_side_mu;                 // held from fork to join of one enqueue
std::map<int, SideStreams> g_side;

hipError_t side_streams(SideStreams **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  SideStreams &ss = g_side[dev];
  if (!ss.fork) {
    for (int k = 1; k < kMaxGroups && e == hipSuccess; ++k) {
      e = hipStreamCreateWithFlags(&ss.s[k], hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&ss.join[k], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming);
    if (e != hipSuccess) return e;
  }
  *out = &ss;
  return hipSuccess;
}

hipError_t launch_group(const BatchPlan &bp, const lsaw::BatchLaunch &b, size_t k, int grid,
                        hipStream_t st) {
  return bp.full ? lsaw::launch_full_batch(b, bp.groups[k].variant, grid, st)
                 : lsaw::launch_batch(b, bp.groups[k].variant, grid, st);
}

// Enqueue every group of a batch on `st`.  Concurrent: group 0 on st itself,
// the others forked onto side streams and joined back, each on its own range
// of arena slices (one group's tail overlaps another's work).  Otherwise the
// groups run one after another on st, all from slice 0.  Works under stream
// capture.
hipError_t enqueue_groups(const BatchPlan &bp, uint8_t *ws, const std::vector<int> &grids,
                          bool concurrent, hipStream_t st) {
  if (bp.groups.empty()) return hipSuccess;
  if (bp.groups.size() == 1 || !concurrent) {
    hipError_t e = hipSuccess;
    for (size_t k = 0; k < bp.groups.size() && e == hipSuccess; ++k) {
      lsaw::BatchLaunch b = batch_launch(bp, ws, k);
      e = lsaw::launch_batch_reset(b.counter, st);
      if (e == hipSuccess) e = launch_group(bp, b, k, grids[k], st);
    }
    return e;
  }
  std::lock_guard<std::mutex> lk(g_side_mu);
  SideStreams *ss = nullptr;
  hipError_t e = side_streams(&ss);
  if (e == hipSuccess) e = hipEventRecord(ss->fork, st);
  uint64_t first = 0;
  for (size_t k = 0; k < bp.groups.size() && e == hipSuccess; ++k) {
    hipStream_t gs = k == 0 ? st : ss->s[k];
    if (k > 0) e = hipStreamWaitEvent(gs, ss->fork, 0);
    lsaw::BatchLaunch b = batch_launch(bp, ws, k);
    b.arena += first * bp.arena_bytes;            // disjoint arena slices per group
    first += (uint64_t)grids[k];
    if (e == hipSuccess) e = lsaw::launch_batch_reset(b.counter, gs);
    if (e == hipSuccess) e = launch_group(bp, b, k, grids[k], gs);
    if (e == hipSuccess && k > 0) e = hipEventRecord(ss->join[k], gs);
  }
  for (size_t k = 1; k < bp.groups.size() && e == hipSuccess; ++k) e = hipStreamWaitEvent(st, ss->join[k], 0);
  return e;
}

}  // namespace

namespace {

// Work lists of labs_walks_batch go to the device through a ring of pinned
// host buffers per device, so the copy is truly asynchronous and the call
// returns without waiting on the caller's stream.  A slot is reused only
// after its previous copy has completed (an event per slot); a slot grows
// (pinned allocation) only when a list is larger than any it held before.
constexpr int kStageSlots = 4;
struct StageRing {
  void *host[kStageSlots] = {nullptr};
  size_t cap[kStageSlots] = {0};
  hipEvent_t done[kStageSlots] = {nullptr};
  bool used[kStageSlots] = {false};
  int next = 0;
};
std::mutex g_stage_mu;
std::map<int, StageRing> g_stage;

// Copies the byte ranges (src[i], n[i]) to dst[i] on `st` through one slot.
hipError_t upload_async(int count, void *const *dst, const void *const *src, const size_t *n,
                        hipStream_t st) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_stage_mu);
  StageRing &ring = g_stage[dev];
  const int k = ring.next;
  ring.next = (k + 1) % kStageSlots;
  if (!ring.done[k]) {
    e = hipEventCreateWithFlags(&ring.done[k], hipEventDisableTiming);
    if (e != hipSuccess) return e;
  }
  if (ring.used[k]) {
    e = hipEventSynchronize(ring.done[k]);      // the slot's previous copy has been read
    if (e != hipSuccess) return e;
  }
  size_t total = 0;
  for (int i = 0; i < count; ++i) total += (n[i] + 255) & ~(size_t)255;
  if (ring.cap[k] < total) {
    if (ring.host[k]) (void)hipHostFree(ring.host[k]);
    ring.host[k] = nullptr;
    ring.cap[k] = 0;
    const size_t want = std::max<size_t>(total, (size_t)1 << 16);
    e = hipHostMalloc(&ring.host[k], want, hipHostMallocDefault);
    if (e != hipSuccess) return e;
    ring.cap[k] = want;
  }
  uint8_t *h = static_cast<uint8_t *>(ring.host[k]);
  size_t off = 0;
  for (int i = 0; i < count && e == hipSuccess; ++i) {
    if (n[i] == 0) continue;
    memcpy(h + off, src[i], n[i]);
    e = hipMemcpyAsync(dst[i], h + off, n[i], hipMemcpyHostToDevice, st);
    off += (n[i] + 255) & ~(size_t)255;
  }
  if (e == hipSuccess) e = hipEventRecord(ring.done[k], st);
  ring.used[k] = e == hipSuccess;
  return e;
}

}  // namespace

struct labs_batch_graph {
  hipGraph_t graph;
  hipGraphExec_t exec;
};

extern "C" {

}  // extern "C"

namespace {

int32_t batch_workspace_bytes(const labs_instance *inst, int32_t n_inst, uint64_t *bytes, bool full) {
  if (!bytes) return fail(LABS_EINVAL, "NULL bytes");
  BatchPlan bp;
  int32_t rc = plan_batch(inst, n_inst, bp, full);
  if (rc != LABS_OK) return rc;
  // Groups one after another: the largest group's grid of arena slices.
  // (A workspace with a slice for every workgroup of every group lets the
  // groups run concurrently; see labs_batch_workspace_bytes in labs.h.)
  int64_t g = 1;
  for (const BatchGroup &grp : bp.groups) {
    int64_t resident = 0;
    rc = device_resident_blocks(grp.variant, bp.full, &resident);
    if (rc != LABS_OK) return rc;
    g = std::max<int64_t>(g, std::min<int64_t>(grp.count, resident));
  }
  *bytes = bp.arena_off + (uint64_t)g * bp.arena_bytes;
  return ok();
}

int32_t walks_batch(const labs_instance *inst, int32_t n_inst, void *workspace, uint64_t ws_bytes,
                    void *stream, bool full) {
  BatchPlan bp;
  int32_t rc = plan_batch(inst, n_inst, bp, full);
  if (rc != LABS_OK) return rc;
  if (bp.items.empty()) return ok();
  if (!workspace) return fail(LABS_EINVAL, "NULL workspace");
  std::vector<int> grids;
  bool concurrent = false;
  rc = batch_grids(bp, ws_bytes, grids, &concurrent);
  if (rc != LABS_OK) return rc;
  uint8_t *ws = static_cast<uint8_t *>(workspace);
  hipStream_t st = as_stream(stream);
  void *dst[2] = {ws + bp.items_off, ws + bp.inst_off};
  const void *src[2] = {bp.items.data(), bp.inst.data()};
  const size_t nb[2] = {bp.items.size() * sizeof(lsaw::BatchItemDev),
                        bp.inst.size() * sizeof(lsaw::BatchInstanceDev)};
  hipError_t e = upload_async(2, dst, src, nb, st);
  if (e == hipSuccess) e = enqueue_groups(bp, ws, grids, concurrent, st);
  if (e != hipSuccess) return fail(LABS_EDEVICE, "batch launch: %s", hipGetErrorString(e));
  return ok();
}

}  // namespace

extern "C" {

int32_t labs_batch_workspace_bytes(const labs_instance *inst, int32_t n_inst, uint64_t *bytes) {
  return batch_workspace_bytes(inst, n_inst, bytes, false);
}

int32_t labs_walks_batch(const labs_instance *inst, int32_t n_inst, void *workspace,
                         uint64_t ws_bytes, void *stream) {
  return walks_batch(inst, n_inst, workspace, ws_bytes, stream, false);
}

int32_t labs_full_batch_workspace_bytes(const labs_instance *inst, int32_t n_inst, uint64_t *bytes) {
  return batch_workspace_bytes(inst, n_inst, bytes, true);
}

int32_t labs_full_walks_batch(const labs_instance *inst, int32_t n_inst, void *workspace,
                              uint64_t ws_bytes, void *stream) {
  return walks_batch(inst, n_inst, workspace, ws_bytes, stream, true);
}

int32_t labs_batch_graph_create(const labs_instance *inst, int32_t n_inst, void *workspace,
                                uint64_t ws_bytes, labs_batch_graph **graph) {
  if (!graph) return fail(LABS_EINVAL, "NULL graph");
  *graph = nullptr;
  BatchPlan bp;
  int32_t rc = plan_batch(inst, n_inst, bp);
  if (rc != LABS_OK) return rc;
  if (!workspace) return fail(LABS_EINVAL, "NULL workspace");
  std::vector<int> grids;
  bool concurrent = false;
  if (!bp.groups.empty()) {
    rc = batch_grids(bp, ws_bytes, grids, &concurrent);
    if (rc != LABS_OK) return rc;
  }
  uint8_t *ws = static_cast<uint8_t *>(workspace);
  hipError_t e = hipSuccess;
  if (!bp.items.empty()) {
    e = hipMemcpy(ws + bp.items_off, bp.items.data(), bp.items.size() * sizeof(lsaw::BatchItemDev),
                  hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(ws + bp.inst_off, bp.inst.data(), bp.inst.size() * sizeof(lsaw::BatchInstanceDev),
                    hipMemcpyHostToDevice);
  }
  hipStream_t cs = nullptr;
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  labs_batch_graph *g = new labs_batch_graph{nullptr, nullptr};
  if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    // a reset kernel (not a memset node) before every group's launch
    hipError_t k = enqueue_groups(bp, ws, grids, concurrent, cs);
    e = hipStreamEndCapture(cs, &g->graph);
    if (e == hipSuccess) e = k;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (cs) (void)hipStreamDestroy(cs);
  if (e != hipSuccess) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return fail(LABS_EDEVICE, "graph capture: %s", hipGetErrorString(e));
  }
  *graph = g;
  return ok();
}

int32_t labs_batch_graph_launch(labs_batch_graph *graph, void *stream) {
  if (!graph) return fail(LABS_EINVAL, "NULL graph");
  hipError_t e = hipGraphLaunch(graph->exec, as_stream(stream));
  if (e != hipSuccess) return fail(LABS_EDEVICE, "graph launch: %s", hipGetErrorString(e));
  return ok();
}

int32_t labs_batch_graph_destroy(labs_batch_graph *graph) {
  if (!graph) return ok();
  if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
  if (graph->graph) (void)hipGraphDestroy(graph->graph);
  delete graph;
  return ok();
}

int32_t labs_tune_set(int32_t L, int32_t lanes_per_walk, double load_factor) {
  if (!valid_skew_L(L)) return fail(LABS_EINVAL, "L=%d: need odd L with 3 <= L <= %d", L, lsaw::kLMax);
  if (lanes_per_walk != 1 && lanes_per_walk != 2 && lanes_per_walk != 4 && lanes_per_walk != 8)
    return fail(LABS_EINVAL, "lanes_per_walk=%d: use 1, 2, 4 or 8", lanes_per_walk);
  if (!(load_factor > 0.0 && load_factor <= 0.9))
    return fail(LABS_EINVAL, "load_factor=%g: use a value in (0, 0.9]", load_factor);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[L] = Tuned{lanes_per_walk, load_factor};
  return ok();
}

int32_t labs_tune_get(int32_t L, int32_t *lanes_per_walk, double *load_factor) {
  if (!valid_skew_L(L)) return fail(LABS_EINVAL, "L=%d: need odd L with 3 <= L <= %d", L, lsaw::kLMax);
  bool found;
  Tuned t;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(L);
    found = it != g_tune.end();
    t = found ? it->second : Tuned{4, 0.5};
  }
  if (lanes_per_walk) *lanes_per_walk = t.lanes;
  if (load_factor) *load_factor = t.load_factor;
  if (!found) {
    g_err = "no tuned entry";
    return LABS_ENOTFOUND;
  }
  return ok();
}

int32_t labs_autotune(int32_t L, int64_t n_walks, int64_t walk_len, void *workspace,
                      uint64_t ws_bytes, void *stream, int32_t *best_lanes, double *best_load_factor) {
  if (!valid_skew_L(L)) return fail(LABS_EINVAL, "L=%d: need odd L with 3 <= L <= %d", L, lsaw::kLMax);
  if (n_walks <= 0 || walk_len <= 0) return fail(LABS_EINVAL, "autotune needs n_walks > 0 and walk_len > 0");
  if (!workspace) return fail(LABS_EINVAL, "NULL workspace");
  labs_plan base{2, 0.5, 0};
  uint64_t need = 0;
  int32_t rc = labs_walks_workspace_bytes(L, n_walks, walk_len, &base, &need);
  if (rc != LABS_OK) return rc;
  const int W = lsaw::key_words_for(L);
  // Result buffers of the timing runs sit at the front of the workspace.
  const uint64_t res_bytes = align256((uint64_t)n_walks * (8u * W + 12u));
  if (ws_bytes < need + res_bytes)
    return fail(LABS_EINVAL, "autotune workspace below %llu bytes", (unsigned long long)(need + res_bytes));
  hipStream_t st = as_stream(stream);
  uint8_t *ws = static_cast<uint8_t *>(workspace);
  uint64_t *best_seq = reinterpret_cast<uint64_t *>(ws);
  int64_t *steps = reinterpret_cast<int64_t *>(ws + (uint64_t)n_walks * 8u * W);
  int32_t *best_E = reinterpret_cast<int32_t *>(ws + (uint64_t)n_walks * (8u * W + 8u));
  void *tables = ws + res_bytes;
  const uint64_t tables_bytes = ws_bytes - res_bytes;
  hipError_t e = hipSuccess;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  e = hipEventCreate(&t0);
  if (e == hipSuccess) e = hipEventCreate(&t1);
  float best_ms = 1e30f;
  Tuned best{4, 0.5};
  const int lanes[3] = {2, 4, 8};
  const double lfs[2] = {0.5, 0.67};
  for (int li = 0; li < 3 && e == hipSuccess; ++li) {
    for (int fi = 0; fi < 2 && e == hipSuccess; ++fi) {
      // Timed on the persistent batch kernel (one instance), which runs the
      // batches and served requests the table is for; the batch uses as many
      // resident workgroups as the workspace has table slices for.
      labs_instance in{};
      in.L = L;
      in.lanes_per_walk = lanes[li];
      in.n_walks = n_walks;
      in.walk_len = walk_len;
      in.starts = nullptr;
      in.load_factor = lfs[fi];
      in.out = labs_walk_out{best_seq, best_E, steps, nullptr, nullptr, nullptr, 0};
      // one untimed run (clock ramp), one timed run
      for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
        in.seed = 1234 + rep;
        if (rep == 1) e = hipEventRecord(t0, st);
        if (e != hipSuccess) break;
        rc = labs_walks_batch(&in, 1, tables, tables_bytes, stream);
        if (rc != LABS_OK) { e = hipErrorUnknown; break; }
        if (rep == 1) e = hipEventRecord(t1, st);
      }
      if (e == hipSuccess) e = hipEventSynchronize(t1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
      if (e == hipSuccess && ms < best_ms) { best_ms = ms; best = Tuned{lanes[li], lfs[fi]}; }
    }
  }
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  if (e != hipSuccess) return fail(LABS_EDEVICE, "autotune: %s", rc != LABS_OK ? g_err.c_str() : hipGetErrorString(e));
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[L] = best;
  }
  if (best_lanes) *best_lanes = best.lanes;
  if (best_load_factor) *best_load_factor = best.load_factor;
  return ok();
}

}  // extern "C"

namespace lsaw {

int32_t set_error(int32_t code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int32_t clear_error() { return ok(); }

bool table_geometry(int32_t L, int64_t walk_len, double load_factor, uint32_t *n_buckets,
                    uint64_t *table_bytes, bool full) {
  labs_plan lp{full ? 0 : 2, load_factor, 0};
  Plan p;
  if ((full ? make_full_plan(L, walk_len, &lp, p) : make_plan(L, walk_len, &lp, p)) != LABS_OK) return false;
  *n_buckets = p.n_buckets;
  *table_bytes = p.table_bytes;
  return true;
}

void tuned_plan(int32_t L, int32_t *lanes, double *load_factor) {
  const Tuned t = tuned_for(L);
  *lanes = t.lanes;
  *load_factor = t.load_factor;
}

}  // namespace lsaw
