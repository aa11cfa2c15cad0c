// labs_device.h -- device helpers shared by the walk kernels of liblabs.so
// (skew-symmetric space and whole space): bit and lane-exchange primitives,
// the exact visited table with its incremental hash, and the per-lane top-K.
// Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>
#include "labs_internal.h"

namespace lsaw {

template <int I, int N, class F>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// v[i] for a small register array and a runtime index (select chain, no scratch).
template <int N>
__device__ __forceinline__ uint32_t sel(const uint32_t (&v)[N], int i) {
  uint32_t r = v[0];
#pragma unroll
  for (int k = 1; k < N; ++k) r = (i == k) ? v[k] : r;
  return r;
}

// ---------------------------------------------------------------------------
// Small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ uint32_t popc_add(uint32_t x, uint32_t acc) {
  uint32_t r;
  asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(acc));
  return r;
}

// Median of three unsigned values (one v_med3_u32).
__device__ __forceinline__ uint32_t umed3(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t r;
  asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}

// (a << S) + b as one v_lshl_add_u32 (kept as a chain, not reassociated).
template <int S>
__device__ __forceinline__ uint32_t lshl_add(uint32_t a, uint32_t b) {
  uint32_t r;
  asm("v_lshl_add_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "I"(S), "v"(b));
  return r;
}

// a * M + b on the 24-bit signed multiplier (one v_mad_i32_i24); |a| < 2^23.
template <int M>
__device__ __forceinline__ uint32_t mad_i24(uint32_t a, uint32_t b) {
  uint32_t r;
  asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "i"(M), "v"(b));
  return r;
}

__device__ __forceinline__ uint32_t funnel(uint32_t hi, uint32_t lo, uint32_t sh) {
  return __builtin_amdgcn_alignbit(hi, lo, sh);
}

// Issue priority of a wavefront (s_setprio, 0..3) by the phase of its walk
// step.  When several waves of a SIMD are ready, the higher priority issues
// first; a wave is raised as its scan nears the end and while it issues a
// visited-table probe, and lowered for the move, so a wave's HBM round trip
// starts as early as possible and overlaps the other waves' scans.  Whether
// that beats issuing by age depends on the kernel's shape, so it is used
// where it measured faster (65,536 walks per length, with and without, on
// one GPU): skew-symmetric walk kernels with 1, 2, 3 or 6 lag words (+3 to
// +14 %; 4 and 5 words lost 4-5 %), whole-space walk kernels with 2, 3, 4,
// 7 or 8 words (+3 to +14 %; 1, 5 and 6 words lost 3-5 %).  The persistent
// batch kernels issue by age (the schedule measured 1-7 % slower there).
enum : int { kPrioMove = 0, kPrioResolve = 1, kPrioScanEarly = 1, kPrioScanLate = 2, kPrioProbe = 3 };
constexpr bool kBatchPriority = false;
constexpr bool walk_priority(int nw) { return nw <= 3 || nw == 6; }
constexpr bool full_walk_priority(int nw) { return (nw >= 2 && nw <= 4) || nw >= 7; }

template <int P, bool kOn>
__device__ __forceinline__ void issue_priority() {
  if constexpr (kOn) __builtin_amdgcn_s_setprio(P);
}

// Priority at the start of scan run sr of nruns: early, late, then the last
// run (whose end is the probe) at the probe's level.
template <bool kOn>
__device__ __forceinline__ void scan_run_priority(int sr, int nruns) {
  if constexpr (kOn) {
    if (sr == nruns - 1) issue_priority<kPrioProbe, true>();
    else if (sr == 1) issue_priority<kPrioScanLate, true>();
  }
}

// Min / max over the G consecutive lanes that cooperate on one walk, with DPP
// lane exchanges inside the VALU (no LDS round trip): quad permutations swap
// neighbours and pairs within each group of four lanes, and the half-row
// mirror (lane i <-> 7 - i within eight lanes) joins two quads.
constexpr int kDppQuadSwap1 = 0xB1;      // quad_perm [1, 0, 3, 2]
constexpr int kDppQuadSwap2 = 0x4E;      // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141;    // row_half_mirror

template <int CTRL>
__device__ __forceinline__ uint32_t dpp(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}
template <int G>
__device__ __forceinline__ uint32_t group_min(uint32_t v) {
  if constexpr (G >= 2) v = min(v, dpp<kDppQuadSwap1>(v));
  if constexpr (G >= 4) v = min(v, dpp<kDppQuadSwap2>(v));
  if constexpr (G >= 8) v = min(v, dpp<kDppHalfMirror>(v));
  return v;
}
template <int G>
__device__ __forceinline__ uint32_t group_max(uint32_t v) {
  if constexpr (G >= 2) v = max(v, dpp<kDppQuadSwap1>(v));
  if constexpr (G >= 4) v = max(v, dpp<kDppQuadSwap2>(v));
  if constexpr (G >= 8) v = max(v, dpp<kDppHalfMirror>(v));
  return v;
}
// Same with the group size known only at run time (G == 0), wave-uniform Gl.
template <int G>
__device__ __forceinline__ uint32_t grp_min(uint32_t v, int Gl) {
  if constexpr (G > 0) {
    return group_min<G>(v);
  } else {
    if (Gl >= 2) v = min(v, dpp<kDppQuadSwap1>(v));
    if (Gl >= 4) v = min(v, dpp<kDppQuadSwap2>(v));
    if (Gl >= 8) v = min(v, dpp<kDppHalfMirror>(v));
    return v;
  }
}
template <int G>
__device__ __forceinline__ uint32_t grp_max(uint32_t v, int Gl) {
  if constexpr (G > 0) {
    return group_max<G>(v);
  } else {
    if (Gl >= 2) v = max(v, dpp<kDppQuadSwap1>(v));
    if (Gl >= 4) v = max(v, dpp<kDppQuadSwap2>(v));
    if (Gl >= 8) v = max(v, dpp<kDppHalfMirror>(v));
    return v;
  }
}

__host__ __device__ constexpr int clog2(int v) { int b = 0; while ((1 << b) < v) ++b; return b; }

__device__ __forceinline__ uint32_t prefix_mask(int n, int w) {
  const int len = n - 32 * w;
  return len >= 32 ? 0xFFFFFFFFu : (len <= 0 ? 0u : ((1u << len) - 1u));
}

constexpr uint32_t kKeyMax = 0xFFFFFFFFu;
constexpr int32_t kBias = 1 << 23;      // bias of the scaled energy change inside a candidate key

// ---------------------------------------------------------------------------
// Visited table
// ---------------------------------------------------------------------------
// A packed key of up to 255 bits (bit b in word b / 64).
struct Key { uint64_t w0, w1, w2, w3; };

// Bucket of a key: an XOR-linear (Zobrist) hash -- the XOR of one random
// 32-bit word per set key bit -- mapped onto [0, n_buckets) by a
// multiply-high.  A walk keeps the hash of its pivot, so the hash of any
// neighbour is one XOR away.  The table stores full keys, so the hash only
// decides where a key is looked for, never whether it is found.
__device__ __forceinline__ uint32_t zobrist_word(int jm1) {
  return (uint32_t)(mix64(0xA0761D6478BD642Full + (uint64_t)jm1) >> 32);
}
__device__ __forceinline__ uint32_t bucket_of_hash(uint32_t h, uint32_t n_buckets) {
  return __umulhi(h, n_buckets);
}

// One bucket is one 128-byte line: a probe reads the whole line it fetches
// from HBM.  Entry formats (keys of at most 95 / 127 / 191 bits):
//   kE12: 10 entries of 12 bytes at dwords 3e..3e+2 (key bits 0-31, 32-63,
//         64-94 with bit 31 of the third dword set when the entry is used);
//         dword 31 holds the number of entries in the bucket;
//   kE16: 8 entries of 16 bytes (key bits 0-126, bit 127 set when used);
//   kE32: 4 entries of 32 bytes (key bits 0-254, bit 255 set when used).
// Entries fill in order and are never deleted, so a present key lies before
// the first free entry.
struct Bucket { uint4 q[8]; };

__device__ __forceinline__ Bucket load_bucket(const uint8_t *bucket) {
  const uint4 *p = reinterpret_cast<const uint4 *>(bucket);
  Bucket b;
#pragma unroll
  for (int i = 0; i < 8; ++i) b.q[i] = p[i];
  return b;
}

// Dword i of a loaded bucket (i a compile-time constant after unrolling).
__device__ __forceinline__ uint32_t bucket_dword(const Bucket &b, int i) {
  const uint4 &v = b.q[i >> 2];
  return (i & 3) == 0 ? v.x : (i & 3) == 1 ? v.y : (i & 3) == 2 ? v.z : v.w;
}

// Test one loaded bucket in format fmt, one of [FLO, FHI] (the formats the
// caller's lengths can meet).  Returns 2 = key present, 1 = absent (n = index
// of the first free entry), 0 = bucket full without the key.  No early exits:
// every entry is compared.
template <int FLO, int FHI>
__device__ __forceinline__ int test_bucket(const Bucket &bk, const Key &k, int fmt, uint32_t &n) {
  const uint32_t k0 = (uint32_t)k.w0, k1 = (uint32_t)(k.w0 >> 32);
  const uint32_t k2 = (uint32_t)k.w1, k3 = (uint32_t)(k.w1 >> 32);
  bool found = false;
  uint32_t cnt = 0u, cap = 1u;
  if constexpr (FLO <= kE12 && kE12 <= FHI) {
    if (fmt == kE12) {
      const uint32_t k2f = k2 | 0x80000000u;
#pragma unroll
      for (int e = 0; e < 10; ++e) {
        const uint32_t x = (bucket_dword(bk, 3 * e) ^ k0) | (bucket_dword(bk, 3 * e + 1) ^ k1) |
                           (bucket_dword(bk, 3 * e + 2) ^ k2f);
        found = found || x == 0u;
      }
      cnt = bucket_dword(bk, 31);
      cap = 10u;
    }
  }
  if constexpr (FLO <= kE16 && kE16 <= FHI) {
    if (fmt == kE16) {
      const uint32_t k3f = k3 | 0x80000000u;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const uint32_t x = (bucket_dword(bk, 4 * e) ^ k0) | (bucket_dword(bk, 4 * e + 1) ^ k1) |
                           (bucket_dword(bk, 4 * e + 2) ^ k2) | (bucket_dword(bk, 4 * e + 3) ^ k3f);
        found = found || x == 0u;
        cnt += bucket_dword(bk, 4 * e + 3) >> 31;
      }
      cap = 8u;
    }
  }
  if constexpr (FLO <= kE32 && kE32 <= FHI) {
    if (fmt == kE32) {
      const uint32_t k4 = (uint32_t)k.w2, k5 = (uint32_t)(k.w2 >> 32);
      const uint32_t k6 = (uint32_t)k.w3, k7f = (uint32_t)(k.w3 >> 32) | 0x80000000u;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint32_t x = (bucket_dword(bk, 8 * e) ^ k0) | (bucket_dword(bk, 8 * e + 1) ^ k1) |
                           (bucket_dword(bk, 8 * e + 2) ^ k2) | (bucket_dword(bk, 8 * e + 3) ^ k3) |
                           (bucket_dword(bk, 8 * e + 4) ^ k4) | (bucket_dword(bk, 8 * e + 5) ^ k5) |
                           (bucket_dword(bk, 8 * e + 6) ^ k6) | (bucket_dword(bk, 8 * e + 7) ^ k7f);
        found = found || x == 0u;
        cnt += bucket_dword(bk, 8 * e + 7) >> 31;
      }
      cap = 4u;
    }
  }
  n = cnt;
  return found ? 2 : (cnt < cap ? 1 : 0);
}

template <int FLO, int FHI>
__device__ __forceinline__ int scan_bucket(const uint8_t *bucket, const Key &k, int fmt, uint32_t &n) {
  return test_bucket<FLO, FHI>(load_bucket(bucket), k, fmt, n);
}

// Stores key k as entry n of a bucket (n = the first free entry found by its probe).
template <int FLO, int FHI>
__device__ __forceinline__ void store_entry(uint8_t *bucket, uint32_t n, const Key &k, int fmt) {
  if constexpr (FLO <= kE12 && kE12 <= FHI) {
    if (fmt == kE12) {
      uint32_t *d = reinterpret_cast<uint32_t *>(bucket);
      d[3 * n] = (uint32_t)k.w0;
      d[3 * n + 1] = (uint32_t)(k.w0 >> 32);
      d[3 * n + 2] = (uint32_t)k.w1 | 0x80000000u;
      d[31] = n + 1u;
    }
  }
  if constexpr (FLO <= kE16 && kE16 <= FHI) {
    if (fmt == kE16) {
      uint4 v;
      v.x = (uint32_t)k.w0; v.y = (uint32_t)(k.w0 >> 32);
      v.z = (uint32_t)k.w1; v.w = (uint32_t)(k.w1 >> 32) | 0x80000000u;
      reinterpret_cast<uint4 *>(bucket)[n] = v;
    }
  }
  if constexpr (FLO <= kE32 && kE32 <= FHI) {
    if (fmt == kE32) {
      uint4 a, b;
      a.x = (uint32_t)k.w0; a.y = (uint32_t)(k.w0 >> 32);
      a.z = (uint32_t)k.w1; a.w = (uint32_t)(k.w1 >> 32);
      b.x = (uint32_t)k.w2; b.y = (uint32_t)(k.w2 >> 32);
      b.z = (uint32_t)k.w3; b.w = (uint32_t)(k.w3 >> 32) | 0x80000000u;
      reinterpret_cast<uint4 *>(bucket)[2 * n] = a;
      reinterpret_cast<uint4 *>(bucket)[2 * n + 1] = b;
    }
  }
}

__device__ __forceinline__ Key flip_key(const Key &k, uint32_t jm1) {
  Key r = k;
  const uint64_t bit = 1ull << (jm1 & 63u);
  const uint32_t w = jm1 >> 6;
  r.w0 ^= (w == 0) ? bit : 0ull;
  r.w1 ^= (w == 1) ? bit : 0ull;
  r.w2 ^= (w == 2) ? bit : 0ull;
  r.w3 ^= (w == 3) ? bit : 0ull;
  return r;
}

// flip_key for keys of at most KWM words (higher words stay as they are).
template <int KWM>
__device__ __forceinline__ Key flip_key_n(const Key &k, uint32_t jm1) {
  if constexpr (KWM >= 4) {
    return flip_key(k, jm1);
  } else if constexpr (KWM == 3) {
    Key r = k;
    const uint64_t bit = 1ull << (jm1 & 63u);
    const uint32_t w = jm1 >> 6;
    r.w0 ^= (w == 0) ? bit : 0ull;
    r.w1 ^= (w == 1) ? bit : 0ull;
    r.w2 ^= (w == 2) ? bit : 0ull;
    return r;
  } else {
    Key r = k;
    const uint64_t bit = 1ull << (jm1 & 63u);
    if constexpr (KWM == 1) {
      r.w0 ^= bit;
    } else {
      const bool hi = (jm1 >> 6) != 0u;
      r.w0 ^= hi ? 0ull : bit;
      r.w1 ^= hi ? bit : 0ull;
    }
    return r;
  }
}

__device__ __forceinline__ uint32_t key_bit(const Key &k, int jm1) {
  const uint64_t w = (jm1 >> 6) == 0 ? k.w0 : (jm1 >> 6) == 1 ? k.w1 : (jm1 >> 6) == 2 ? k.w2 : k.w3;
  return (uint32_t)((w >> (jm1 & 63)) & 1ull);
}

template <int K>
__device__ __forceinline__ void topk_insert(uint32_t (&tk)[K], uint32_t x) {
  if constexpr (K == 1) {
    tk[0] = min(tk[0], x);
  } else {
    // Sorted insertion: new[i] = median(old[i-1], old[i], x), new[0] = min.
#pragma unroll
    for (int i = K - 1; i >= 1; --i) tk[i] = umed3(tk[i - 1], tk[i], x);   // tk sorted
    tk[0] = min(tk[0], x);
  }
}

}  // namespace lsaw
