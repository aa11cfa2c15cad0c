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

int32_t make_plan(int32_t L, int64_t walk_len, const labs_plan *p, Plan &out) {
  if (!valid_skew_L(L)) return fail(LABS_EINVAL, "L=%d: need odd L with 3 <= L <= %d", L, lsaw::kLMax);
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
  const int epb = lsaw::kBucketBytes / lsaw::entry_bytes_for(L);
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
    w.tables = static_cast<uint8_t *>(workspace);
    w.table_bytes = p.table_bytes;
    w.n_buckets = p.n_buckets;
    w.lanes_per_walk = G;
    hipError_t e = lsaw::launch_walks(w, st);
    if (e != hipSuccess) return fail(LABS_EDEVICE, "walk launch: %s", hipGetErrorString(e));
  }
  return ok();
}

}  // extern "C"
