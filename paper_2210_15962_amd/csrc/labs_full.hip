// labs_full.hip -- gfx950 walk kernel of liblabs.so over the whole search
// space of the LABS problem: all 2^L binary sequences of any length L, a
// neighbour negating one of the L positions (the sokol_full solver that
// Boskovic, Herzog & Brest, arXiv 2210.15962, Sec. 5, name as future work).
// The walk rules are those of Eq. 3 and Alg. 2: move to the unvisited
// neighbour of lowest energy, ties to the lowest position, stop when every
// neighbour has been visited, track the best with a strict "<".
//
// Notation: s_1..s_L, lags k = 1..L-1 at lag index t = k-1 (32 lags per lag
// word), C_k of Eq. 1.  Negating s_i changes C_k by 2 u_k with
//     u_k = -s_i (F_k s_{i+k} + B_k s_{i-k}),  F_k = [k <= L-i], B_k = [k < i],
// so that
//     dE_i = 4 sum_k u_k C_k + 4 sum_k u_k^2,
//     sum_k u_k^2 = (L-1) + 2 sum_{F and B} s_{i+k} s_{i-k}.
// C_k has the parity p_k of L-k.  The bit planes hold c_k = (C_k - p_k)/2 in
// two's complement; for a sign sigma = +-1 with flag f (1 for -1)
//     sigma C_k = 2 (c_k XOR -f) + 2 f (1 - p_k) + p_k,
// so a signed sum of C over a lag mask costs one XOR/AND/popcount per plane
// word plus one AND/popcount over the even-C lags, whose mask alternates bit
// by bit.  (Derived from Eq. 1.)
//
// Data layout per walk (replicated in each of its lanes):
//   * sequence: two bit arrays in the lane's LDS column, forwards (bit x-1
//     holds f_x) and reversed (bit L-x holds f_x), so the forward and the
//     backward neighbours of any position are one funnel shift away;
//   * c: bit planes in VGPRs, 32 lags per word;
//   * visited set: the exact open-addressing HBM table of the skew-symmetric
//     walks, keyed on the packed sequence (bit i-1 = f_i).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>
#include "labs_internal.h"
#include "labs_device.h"

namespace lsaw {
namespace full {

constexpr int kG = 4;            // lanes per walk
constexpr int kK = 3;            // top-K entries per lane
constexpr int kRunSlots = 32;    // run table: runs (at most 16 occur), then the count in the last slot

// Lag-word class nw holds 32 nw lags, i.e. lengths up to 32 nw + 1; plane
// counts are sized for that bound.  Word w then has |C_k| <= 32 (nw - w), so
// c_k = (C_k - p_k)/2 lies in [-(16 (nw - w) + 1), 16 (nw - w)].
__host__ __device__ constexpr int lclass_max(int nw) { return 32 * nw + 1; }
__host__ __device__ constexpr int planes_of(int nw, int w) {
  return 1 + clog2((lclass_max(nw) - 1 - 32 * w) / 2 + 1);
}
__host__ __device__ constexpr int plane_off(int nw, int w) {
  int s = 0;
  for (int i = 0; i < w; ++i) s += planes_of(nw, i);
  return s;
}

template <int NW>
struct Geom {
  static constexpr int NWB = (NW + 1) / 2;     // words where forward and backward lags overlap
  // Words per bit array: a read of NW + 1 words from any start word of a
  // sequence of at most 32 NW + 1 positions stays inside.
  static constexpr int NWA = 2 * NW + 2;
  static constexpr int LMAX = lclass_max(NW) < kFullLMax ? lclass_max(NW) : kFullLMax;
  static constexpr int DESC = (8 + 2 * NW + NWB + 3) & ~3;   // dwords per row
  static constexpr int NPW = plane_off(NW, NW);
  static constexpr int BMAX = planes_of(NW, 0);
  static constexpr int DROWS = LMAX + 8;       // real rows plus dead rows
  static constexpr int NLOC = (LMAX + kG - 1) / kG;          // candidates per lane
  static constexpr int kSW = (NLOC + 31) / 32;               // sign-mask words
  static constexpr size_t cols_off() { return ((size_t)DROWS * DESC * 4 + 255) & ~(size_t)255; }
  static constexpr size_t runs_off() { return cols_off() + (size_t)2 * NWA * kBlock * 4; }
  static constexpr size_t zob_off() { return runs_off() + kRunSlots * 4; }
  static constexpr size_t lds_bytes() { return zob_off() + (size_t)LMAX * 4; }
};

// Descriptor row of position i (dword offsets).
enum : int {
  FD_FOFF = 0,   // byte offset (within a lane column) of forward source word 0
  FD_FSH = 1,    // funnel shift of the forward vector
  FD_BOFF = 2,
  FD_BSH = 3,
  FD_KC = 4,     // ((((L-1) - 2|F&B| + kBias) << 8) | (i-1)) + 1; dead rows: 0
  FD_KT = 5,     // (nOdd - 2 sum_w 2^(B_w - 1) (|MF_w| + |MB_w|)) << 8, two's complement
  FD_KT8 = 6,    // nOdd << 8 (planes-capped evaluation)
  FD_MASKS = 8   // MF[NW], MB[NW], MFB[NWB]
};

// Column layout: array a (0 forward, 1 reversed), word w, lane l -> dword
// ((a * NWA + w) * kBlock + l).
template <int NW>
__device__ __forceinline__ uint32_t col_word_off(int a, int w) {
  return (uint32_t)(((a * Geom<NW>::NWA + w) * kBlock) * 4);
}

// Lags whose C has even parity (L - k even): bit b of every lag word is lag
// k = 32 w + b + 1, so they are the bits b = L + 1 (mod 2).
__host__ __device__ constexpr uint32_t even_c_mask(int L) { return (L & 1) ? 0x55555555u : 0xAAAAAAAAu; }

template <int NW>
__device__ __forceinline__ void build_descriptors(uint32_t *desc, int L) {
  using Gm = Geom<NW>;
  const uint32_t odd = ~even_c_mask(L);
#pragma unroll 1
  for (int i = 1 + (int)threadIdx.x; i <= L; i += blockDim.x) {
    uint32_t *row = desc + (i - 1) * Gm::DESC;
    const int rb = L - i + 1;                    // reversed-array bit of s_{i-1}
    row[FD_FOFF] = col_word_off<NW>(0, i >> 5);
    row[FD_FSH] = (uint32_t)(i & 31);
    row[FD_BOFF] = col_word_off<NW>(1, rb >> 5);
    row[FD_BSH] = (uint32_t)(rb & 31);
    const int nF = L - i, nB = i - 1;
    int kc = 0, n_odd = 0, n_fb = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      const uint32_t mf = prefix_mask(nF, w), mb = prefix_mask(nB, w);
      row[FD_MASKS + w] = mf;
      row[FD_MASKS + NW + w] = mb;
      if (w < Gm::NWB) row[FD_MASKS + 2 * NW + w] = mf & mb;   // zero past NWB words
      kc += (__builtin_popcount(mf) + __builtin_popcount(mb)) << (planes_of(NW, w) - 1);
      n_odd += __builtin_popcount(mf & odd) + __builtin_popcount(mb & odd);
      n_fb += __builtin_popcount(mf & mb);
    }
    row[FD_KC] = (((uint32_t)(L - 1 - 2 * n_fb + kBias) << 8) | (uint32_t)(i - 1)) + 1u;
    row[FD_KT] = (uint32_t)(n_odd - 2 * kc) << 8;
    row[FD_KT8] = (uint32_t)n_odd << 8;
    row[7] = 0u;
#pragma unroll
    for (int d = FD_MASKS + 2 * NW + Gm::NWB; d < Gm::DESC; ++d) row[d] = 0u;
  }
  // Dead rows L+1 .. L+8: all zero, which gives the key ~0 (never chosen).
  for (int t = (int)threadIdx.x; t < 8 * Gm::DESC; t += blockDim.x) desc[L * Gm::DESC + t] = 0u;
}

// Candidate key of position i: ((dE/4 + kBias) << 8) | (i-1), so unsigned
// order is (dE, i) order.  FW forward and BW backward lag words are formed;
// the caller guarantees that every candidate of the wave has all-zero masks
// past them.  With BP > 0 every word is evaluated on its low BP planes only,
// which is exact when every c of the walk fits BP bits (the caller checks).
//
// Per plane b the count is popcount((c_b XOR f) AND M); the sign plane is
// counted complemented in the full form (so every plane has a positive
// weight and the |M| 2^(B_w - 1) excess is the per-row constant FD_KT).  The
// even-C correction popcount(f AND M AND even) joins plane 0 (weight 1).
template <int NW, int FW, int BW, int BP>
__device__ __forceinline__ uint32_t eval_key(const uint32_t *row, const uint8_t *lds,
                                             uint32_t colbase, const uint32_t *P, uint32_t sg,
                                             uint32_t ev) {
  using Gm = Geom<NW>;
  static_assert(FW >= 0 && FW <= NW && BW >= 0 && BW <= NW, "lag-word counts");
  static_assert(BP == 0 || (BP >= 2 && BP <= planes_of(NW, NW - 1)), "plane cap");
  constexpr int BM = BP > 0 ? BP : Gm::BMAX;
  constexpr int WN = FW > BW ? FW : BW;
  const uint4 d0 = *reinterpret_cast<const uint4 *>(row);
  const uint4 d1 = *reinterpret_cast<const uint4 *>(row + 4);
  const uint32_t *fsrc = reinterpret_cast<const uint32_t *>(lds + colbase + d0.x);
  const uint32_t *bsrc = reinterpret_cast<const uint32_t *>(lds + colbase + d0.z);
  uint32_t fv[FW > 0 ? FW : 1];
  uint32_t bv[BW > 0 ? BW : 1];
  if constexpr (FW > 0) {
    uint32_t lo = fsrc[0];
#pragma unroll
    for (int w = 0; w < FW; ++w) {
      const uint32_t hi = fsrc[(w + 1) * kBlock];
      fv[w] = funnel(hi, lo, d0.y);
      lo = hi;
    }
  }
  if constexpr (BW > 0) {
    uint32_t lo = bsrc[0];
#pragma unroll
    for (int w = 0; w < BW; ++w) {
      const uint32_t hi = bsrc[(w + 1) * kBlock];
      bv[w] = funnel(hi, lo, d0.w);
      lo = hi;
    }
  }
  uint32_t cnt[BM];
#pragma unroll
  for (int b = 0; b < BM; ++b) cnt[b] = 0u;
  uint32_t q = 0u;
  static_for<0, WN>([&](auto wc) {
    constexpr int w = decltype(wc)::value;
    constexpr int off = plane_off(NW, w);
    constexpr int Bw = BP > 0 ? BP : planes_of(NW, w);
    if constexpr (w < FW) {
      const uint32_t mf = row[FD_MASKS + w];
#pragma unroll
      for (int b = 0; b < Bw - 1; ++b) cnt[b] = popc_add((P[off + b] ^ fv[w]) & mf, cnt[b]);
      if constexpr (BP > 0)
        cnt[Bw - 1] = popc_add((P[off + Bw - 1] ^ fv[w]) & mf, cnt[Bw - 1]);
      else
        cnt[Bw - 1] = popc_add(~(P[off + Bw - 1] ^ fv[w]) & mf, cnt[Bw - 1]);
      cnt[0] = popc_add(fv[w] & mf & ev, cnt[0]);
    }
    if constexpr (w < BW) {
      const uint32_t mb = row[FD_MASKS + NW + w];
#pragma unroll
      for (int b = 0; b < Bw - 1; ++b) cnt[b] = popc_add((P[off + b] ^ bv[w]) & mb, cnt[b]);
      if constexpr (BP > 0)
        cnt[Bw - 1] = popc_add((P[off + Bw - 1] ^ bv[w]) & mb, cnt[Bw - 1]);
      else
        cnt[Bw - 1] = popc_add(~(P[off + Bw - 1] ^ bv[w]) & mb, cnt[Bw - 1]);
      cnt[0] = popc_add(bv[w] & mb & ev, cnt[0]);
    }
    if constexpr (w < FW && w < BW && w < Gm::NWB)
      q = popc_add(~(fv[w] ^ bv[w]) & row[FD_MASKS + 2 * NW + w], q);   // |MFB| - count
  });
  uint32_t H, kt;
  if constexpr (BP > 0) {
    // sign plane: weight -2^(BP-1), so the Horner sum opens with
    // cnt[BP-2] - 2 cnt[BP-1]
    H = mad_i24<-2>(cnt[BM - 1], cnt[BM - 2]);
    kt = d1.z;                                   // nOdd << 8
#pragma unroll
    for (int b = BM - 3; b >= 0; --b) H = lshl_add<1>(H, cnt[b]);
  } else {
    H = cnt[BM - 1];                             // complemented sign planes
    kt = d1.y;                                   // (nOdd - 2 Kc) << 8
#pragma unroll
    for (int b = BM - 2; b >= 0; --b) H = lshl_add<1>(H, cnt[b]);
  }
  const uint32_t t = lshl_add<9>(H, kt);        // (sum_F+B sigma C) << 8
  const uint32_t kq = lshl_add<10>(q, d1.x);    // key constant + 4 (|MFB| - q) << 8
  // sg = ~0 when s_i = -1: kq - 1 + t; else kq + ~t = kq - 1 - t.
  return kq + sg + ~(t ^ sg);
}

// Smallest plane cap in {4, 5, 6} valid for every active walk of the wave
// (0: none).  A cap BP is valid for a lane when the planes BP..B_w-1 of every
// lag word equal plane BP-1.
template <int NW>
__device__ __forceinline__ int wave_plane_cap(const uint32_t *P, bool active) {
  uint32_t d4 = 0u, d5 = 0u, d6 = 0u;
  static_for<0, NW>([&](auto wc) {
    constexpr int w = decltype(wc)::value;
    constexpr int off = plane_off(NW, w), Bw = planes_of(NW, w);
#pragma unroll
    for (int b = 4; b < Bw; ++b) {
      const uint32_t d = P[off + b] ^ P[off + b - 1];
      if (b == 4) d4 |= d;
      else if (b == 5) d5 |= d;
      else d6 |= d;
    }
  });
  if (__ballot(active && d6 != 0u) != 0ull) return 0;
  if (__ballot(active && d5 != 0u) != 0ull) return 6;
  if (__ballot(active && d4 != 0u) != 0ull) return 5;
  return 4;
}

// Lag words the candidates of iteration it (i = G it + 1 .. G it + G) need:
// forward words for the smallest i, backward words for the largest.  The
// code is FW * 16 + BW (both at most 8).
__host__ __device__ constexpr int words_of(int it, int L, int G, int nw) {
  const int imin = G * it + 1;
  const int imax = (G * it + G < L) ? G * it + G : L;
  int fw = (L - imin + 31) / 32;
  fw = fw < nw ? fw : nw;
  fw = fw > 0 ? fw : 0;
  int bw = (imax - 1 + 31) / 32;
  bw = bw < nw ? bw : nw;
  return fw * 16 + bw;
}

// Set of codes (0..143) as a 192-bit mask.
struct CodeSet { uint64_t w[3]; };
__host__ __device__ constexpr bool code_in(const CodeSet &m, int c) {
  return c >= 0 && c < 192 && ((m.w[c >> 6] >> (c & 63)) & 1ull) != 0;
}

// Codes the candidate loop of class nw can meet (every length of the class).
__host__ __device__ constexpr CodeSet words_mask(int nw, int G) {
  CodeSet m{{0, 0, 0}};
  const int lo = nw == 1 ? 3 : 32 * (nw - 1) + 2;
  const int hi = (32 * nw + 1) < kFullLMax ? 32 * nw + 1 : kFullLMax;
  for (int L = lo; L <= hi; ++L)
    for (int it = 0; it < (L + G - 1) / G; ++it) {
      const int c = words_of(it, L, G, nw);
      m.w[c >> 6] |= 1ull << (c & 63);
    }
  return m;
}

// Codes of every class in [nlo, nhi] (a batch kernel runs the lengths of
// several classes on the largest one's geometry).
__host__ __device__ constexpr CodeSet words_mask_range(int nlo, int nhi, int G) {
  CodeSet m{{0, 0, 0}};
  for (int c = nlo; c <= nhi; ++c) {
    const CodeSet x = words_mask(c, G);
    for (int i = 0; i < 3; ++i) m.w[i] |= x.w[i];
  }
  return m;
}
template <int NLO, int NHI>
struct ClassCodes { static constexpr CodeSet value = words_mask_range(NLO, NHI, kG); };

// Calls f(FW, BW) as compile-time constants for a wave-uniform code; a code
// outside the kernel's set takes the all-words form, valid for every candidate.
template <int NW, class Codes, class F>
__device__ __forceinline__ void with_words(int code, F &&f) {
  constexpr CodeSet kMask = Codes::value;
  constexpr int kFull = NW * 16 + NW;
  const int eff = code_in(kMask, code) ? code : kFull;
  static_for<0, 16 * NW + NW + 1>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    constexpr int fw = c >> 4, bw = c & 15;
    if constexpr ((code_in(kMask, c) || c == kFull) && fw <= NW && bw <= NW) {
      if (eff == c) f(std::integral_constant<int, fw>{}, std::integral_constant<int, bw>{});
    }
  });
}

// c_k += u_k on the bit planes for the move at position i (u from the
// pre-move neighbour vectors): u_k = -s_i (a_k + b_k), a_k = MF_k ? (f_{i+k}
// ? -1 : 1) : 0, b_k likewise backwards.
template <int NW>
__device__ __forceinline__ void apply_move_planes(const uint32_t *row, const uint8_t *lds,
                                                  uint32_t colbase, uint32_t sbit, uint32_t *P) {
  const uint4 d0 = *reinterpret_cast<const uint4 *>(row);
  const uint32_t *fsrc = reinterpret_cast<const uint32_t *>(lds + colbase + d0.x);
  const uint32_t *bsrc = reinterpret_cast<const uint32_t *>(lds + colbase + d0.z);
  // s_i = +1 -> add -w = ~w + 1; s_i = -1 -> add w.
  const uint32_t ms = sbit ? 0u : 0xFFFFFFFFu;
  uint32_t flo = fsrc[0], blo = bsrc[0];
  static_for<0, NW>([&](auto wc) {
    constexpr int w = decltype(wc)::value;
    constexpr int Bw = planes_of(NW, w), off = plane_off(NW, w);
    const uint32_t fhi = fsrc[(w + 1) * kBlock], bhi = bsrc[(w + 1) * kBlock];
    const uint32_t fv = funnel(fhi, flo, d0.y), bv = funnel(bhi, blo, d0.w);
    flo = fhi;
    blo = bhi;
    const uint32_t a0 = row[FD_MASKS + w], a1 = fv & a0;
    const uint32_t b0 = row[FD_MASKS + NW + w], b1 = bv & b0;
    // w = a + b as 3-bit two's complement (bit 2 is the sign).
    const uint32_t w0 = a0 ^ b0, c1 = a0 & b0;
    const uint32_t t1 = a1 ^ b1;
    const uint32_t w1 = t1 ^ c1;
    const uint32_t c2 = (t1 & c1) | (a1 & b1);
    const uint32_t w2 = t1 ^ c2;
    const uint32_t u0 = w0 ^ ms, u1 = w1 ^ ms, u2 = w2 ^ ms;
    uint32_t carry = ms;
#pragma unroll
    for (int b = 0; b < Bw; ++b) {
      const uint32_t x = (b == 0) ? u0 : (b == 1) ? u1 : u2;
      const uint32_t p = P[off + b];
      // truth tables over (p, x, carry) = (0xF0, 0xCC, 0xAA): 0x96 = XOR3, 0xE8 = majority
      P[off + b] = __builtin_amdgcn_bitop3_b32(p, x, carry, 0x96);
      carry = __builtin_amdgcn_bitop3_b32(p, x, carry, 0xE8);
    }
  });
}

// Waves per SIMD each class is built for (registers capped to fit): four up
// to class 4 (L <= 129), three up to class 7, two for class 8.
template <int NW>
struct FullOccupancy { static constexpr int value = NW <= 4 ? 4 : (NW <= 7 ? 3 : 2); };

// One workgroup's share: up to kBlock / kG walks of one length L.
struct FullTask {
  const uint64_t *starts;   // first pivots of the instance ([walk][KW]) or nullptr
  uint64_t seed;            // seeded starts: SplitMix64 of (seed, walk index)
  int32_t L;
  int32_t n_block;          // walks of this block
  int64_t walk_begin;       // instance index of the block's first walk
  int64_t walk_len;
  uint64_t *best_seq;
  int32_t *best_E;
  int64_t *steps_done;
  uint64_t *digest;
  int16_t *trace_j;
  int32_t *trace_E;
  int64_t n_trace;
  uint32_t *cap_steps;
  uint8_t *tables;          // table of block slot s at tables + s * table_bytes
  uint64_t table_bytes;
  uint32_t n_buckets;
  // serving form only (see the skew-symmetric batch kernel's)
  WalkState *state;         // per-walk progress across launches
  uint8_t *wstat;           // per-walk status: 0 not started, 1 resume, 2 finished
  int64_t step_end;         // a walk stops when it has made this many moves
  const uint32_t *preempt;  // host stop flag polled every 64 moves, or nullptr
  uint32_t *done_flag;      // set to 1 if the block ends with every walk finished
};

// A nonzero stop word from the host (fine-grained memory: read past the
// caches), read by one lane of the wave.
__device__ __forceinline__ bool full_stop_requested(const uint32_t *flag) {
  uint32_t v = 0u;
  if (__lane_id() == 0) v = __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  return __builtin_amdgcn_readfirstlane(v) != 0u;
}

// The walks of one block (geometry of class NW, which serves every shorter
// length too; kFLO the narrowest entry format of the lengths the kernel
// runs; Codes its run codes; kSv the serving form: walks that pause and
// resume across launches).
template <int NW, int kFLO, class Codes, bool kSv = false, bool kPrio = true>
__device__ __forceinline__ void run_full_block(const FullTask &a, uint8_t *lds) {
  using Gm = Geom<NW>;
  constexpr int G = kG, K = kK, lgG = 2;
  static_assert(G == 4, "lane index arithmetic assumes four lanes per walk");
  static_assert(Gm::NLOC <= 64, "one exclusion word per lane");
  uint32_t *desc = reinterpret_cast<uint32_t *>(lds);
  uint8_t *cols = lds + Gm::cols_off();
  uint32_t *runs = reinterpret_cast<uint32_t *>(lds + Gm::runs_off());
  uint32_t *zob = reinterpret_cast<uint32_t *>(lds + Gm::zob_off());

  const int L = a.L;
  const int KW = (L + 63) / 64;
  const int n_block = a.n_block;
  uint8_t *tables = a.tables;

  build_descriptors<NW>(desc, L);
  const int nmax = (L + G - 1) / G;              // candidate-loop iterations
  if (threadIdx.x == 0) {
    // Runs of iterations with equal lag-word counts: (first it << 8) | code,
    // then a sentinel (nmax << 8).  Past kRunSlots - 2 runs the last run takes
    // the all-words form, which serves any candidate.
    int n = 0, prev = -1;
    for (int it = 0; it < nmax; ++it) {
      const int code = words_of(it, L, G, NW);
      if (code == prev) continue;
      if (n == kRunSlots - 2) {
        runs[n - 1] = (runs[n - 1] & ~0xFFu) | (uint32_t)(NW * 16 + NW);
        break;
      }
      runs[n++] = ((uint32_t)it << 8) | (uint32_t)code;
      prev = code;
    }
    runs[n] = (uint32_t)nmax << 8;
    runs[kRunSlots - 1] = (uint32_t)n;
  }
  for (int x = (int)threadIdx.x; x < L; x += blockDim.x) zob[x] = zobrist_word(x);
  const uint4 z = {0u, 0u, 0u, 0u};
  if (kSv && a.wstat) {
    // Walks resumed from an earlier launch keep their tables: clear only the
    // tables of walks that start now.
    const uint64_t n16 = a.table_bytes / 16u;
    for (int sl = 0; sl < n_block; ++sl) {
      if (a.wstat[a.walk_begin + sl] != 0u) continue;      // uniform
      uint4 *p = reinterpret_cast<uint4 *>(tables + (uint64_t)sl * a.table_bytes);
#pragma unroll 4
      for (uint64_t q = threadIdx.x; q < n16; q += kBlock) p[q] = z;
    }
  } else {
    // Clear the visited tables of this block's walks (contiguous, coalesced).
    uint4 *p = reinterpret_cast<uint4 *>(tables);
    const uint64_t n16 = (uint64_t)max(n_block, 0) * (a.table_bytes / 16u);
#pragma unroll 4
    for (uint64_t q = threadIdx.x; q < n16; q += kBlock) p[q] = z;
  }
  __syncthreads();

  const int tid = (int)threadIdx.x;
  const int r = tid % G;                        // lane rank inside the walk group
  const int slot = tid / G;                     // walk slot inside the block
  const int64_t walk = a.walk_begin + slot;
  bool active = slot < n_block;
  // Status of the walk from earlier launches (serving form).
  const uint32_t wst = (kSv && a.wstat && active) ? (uint32_t)a.wstat[walk] : 0u;
  const bool fresh = wst == 0u;                 // starts at P_1 in this launch
  const bool skip = wst == 2u;                  // finished earlier: nothing to do
  if (skip) active = false;
  const uint32_t colbase = (uint32_t)tid * 4u;
  uint32_t *colw = reinterpret_cast<uint32_t *>(cols);
  // visited-table entry format of this length (within the kernel's formats)
  constexpr int kFHI = entry_format(Gm::LMAX);
  const int efmt = entry_format(L);
  const uint32_t ev = even_c_mask(L);
  constexpr int KWM = (Gm::LMAX + 63) / 64;        // key words any length of the class needs

  // ---- first pivot, or the pivot reached by an earlier launch -----------------
  Key P{0, 0, 0};
  WalkState ws{};
  if (active && !fresh) {
    ws = a.state[walk];
    P.w0 = ws.P[0];
    P.w1 = ws.P[1];
    P.w2 = ws.P[2];
    P.w3 = ws.P[3];
  } else if (active) {
    auto start_word = [&](int t) -> uint64_t {
      if (t >= KW) return 0ull;
      uint64_t v;
      if (a.starts) {
        v = a.starts[walk * KW + t];
      } else {
        v = mix64(a.seed + 0x9E3779B97F4A7C15ull * ((uint64_t)walk * (uint64_t)KW + (uint64_t)t + 1u));
      }
      const int bits = L - 64 * t;
      if (bits < 64) v &= ((1ull << bits) - 1ull);
      return v;
    };
    P.w0 = start_word(0);
    P.w1 = start_word(1);
    P.w2 = start_word(2);
    P.w3 = start_word(3);
  }
  if constexpr (KWM < 4) P.w3 = 0;
  if constexpr (KWM < 3) P.w2 = 0;
  if constexpr (KWM < 2) P.w1 = 0;

  // ---- sequence bit arrays ---------------------------------------------------
  for (int w = 0; w < 2 * Gm::NWA; ++w) colw[w * kBlock + tid] = 0u;
#pragma unroll 1
  for (int w = 0; w < (L + 31) / 32; ++w) {
    const uint64_t kw = (w >> 1) == 0 ? P.w0 : (w >> 1) == 1 ? P.w1 : (w >> 1) == 2 ? P.w2 : P.w3;
    colw[w * kBlock + tid] = (uint32_t)(kw >> (32 * (w & 1)));
  }
#pragma unroll 1
  for (int x = 1; x <= L; ++x) {
    if (key_bit(P, x - 1)) {
      const int y = L - x;
      colw[(Gm::NWA + (y >> 5)) * kBlock + tid] |= 1u << (y & 31);
    }
  }

  // ---- C_k (all lags) -> planes of c_k = (C_k - p_k)/2, and E(P_1) -------------
  uint32_t Pl[Gm::NPW];
#pragma unroll
  for (int q = 0; q < Gm::NPW; ++q) Pl[q] = 0u;
  int32_t E = 0;
  static_for<0, NW>([&](auto wc) {
    constexpr int w = decltype(wc)::value;
    constexpr int Bw = planes_of(NW, w), off = plane_off(NW, w);
#pragma unroll 1
    for (int tb = 0; tb < 32; ++tb) {
      const int k = 32 * w + tb + 1;
      if (k >= L) break;
      const int npairs = L - k, q = k >> 5, sh = k & 31;
      int mism = 0;
      for (int ww = 0; 32 * ww < npairs; ++ww) {
        const uint32_t x = colw[ww * kBlock + tid];
        const uint32_t lo = colw[(ww + q) * kBlock + tid];
        const uint32_t hi = colw[(ww + q + 1) * kBlock + tid];
        const uint32_t y = funnel(hi, lo, (uint32_t)sh);
        const int rem = npairs - 32 * ww;
        const uint32_t msk = rem >= 32 ? 0xFFFFFFFFu : ((1u << rem) - 1u);
        mism += __builtin_popcount((x ^ y) & msk);
      }
      const int32_t Ck = npairs - 2 * mism;
      E += Ck * Ck;
      const int32_t ck = (Ck - (npairs & 1)) >> 1;
#pragma unroll
      for (int b = 0; b < Bw; ++b) Pl[off + b] |= (uint32_t)((ck >> b) & 1) << tb;
    }
  });

  int32_t bestE = E;
  Key bestP = P;
  uint64_t h = 0;
  int64_t steps = 0;
  uint32_t prev_im1 = 0xFFFFFFFFu;
  bool trapped = false;
  uint8_t *table = tables + (uint64_t)(active ? slot : 0) * a.table_bytes;
  if (active && !fresh) {
    bestE = ws.bestE;
    bestP = Key{ws.bestP[0], ws.bestP[1], ws.bestP[2], ws.bestP[3]};
    h = ws.h;
    steps = ws.steps;
    prev_im1 = ws.prev_jm1;
    trapped = ws.trapped != 0u;
    if (trapped) active = false;
  }

  uint32_t hP = 0u;
#pragma unroll 1
  for (int x = 0; x < L; ++x) hP ^= key_bit(P, x) ? zob[x] : 0u;

  // Insert P_1 (the table is empty: first entry of its home bucket).
  if (active && fresh && r == 0)
    store_entry<kFLO, kFHI>(table + (uint64_t)bucket_of_hash(hP, a.n_buckets) * kBucketBytes, 0u, P, efmt);

  // Local candidates of lane r: i = r + 1 + G*it; their signs in registers
  // (bit it <-> s_i = -1, 0 past L): the scan reads s_i here, the move toggles it.
  const int ncand = (L - r + G - 1) / G;
  uint32_t smk[Gm::kSW];
#pragma unroll
  for (int w = 0; w < Gm::kSW; ++w) smk[w] = 0u;
#pragma unroll 1
  for (int it = 0; it < nmax; ++it) {
    const int i = r + 1 + G * it;
    const uint32_t bit = i <= L ? key_bit(P, i - 1) : 0u;
    static_for<0, Gm::kSW>([&](auto wc) {
      constexpr int w = decltype(wc)::value;
      if ((it >> 5) == w) smk[w] |= bit << (it & 31);
    });
  }
  auto sign_of = [&](int it) -> uint32_t {      // ~0 if s_i = -1, else 0 (it uniform)
    if constexpr (Gm::kSW == 1) {
      return (uint32_t)__builtin_amdgcn_sbfe((int)smk[0], it & 31, 1);   // it < 32
    } else {
      uint32_t wv = 0u;
      static_for<0, Gm::kSW>([&](auto wc) {
        constexpr int w = decltype(wc)::value;
        wv |= smk[w] & (0u - (uint32_t)((it >> 5) == w));
      });
      return (uint32_t)__builtin_amdgcn_sbfe((int)wv, it & 31, 1);
    }
  };
  const int nruns = (int)__builtin_amdgcn_readfirstlane(runs[kRunSlots - 1]);
  uint32_t ncap4 = 0u, ncap5 = 0u, ncap6 = 0u, ncap0 = 0u;
  const bool tracing = active && walk < a.n_trace;

  // Serving form: a wave makes as many moves as its nearest-to-done walk has
  // left (walks that ran in different waves before may stand at different
  // move counts); walks still short of the end continue in the next launch.
  const int64_t step_stop = kSv ? min(a.step_end, a.walk_len) : a.walk_len;
  int64_t lim = step_stop;
  if constexpr (kSv) {
    if (steps >= step_stop) active = false;
    int64_t rem = active ? step_stop - steps : INT64_MAX;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const int64_t o = __shfl_xor(rem, off);
      rem = o < rem ? o : rem;
    }
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)rem);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)rem >> 32));
    lim = (int64_t)(((uint64_t)hi << 32) | lo);
  }
  for (int64_t step = 0; step < lim; ++step) {
    if (__ballot(active) == 0ull) break;
    if (kSv && a.preempt && (step & 63) == 63 && full_stop_requested(a.preempt)) break;
    // Excluded local candidates (bit it <-> i = r + 1 + G*it): the
    // predecessor, then every candidate found visited during this step.
    uint64_t ex = 0ull;
    if (prev_im1 != 0xFFFFFFFFu && (int)(prev_im1 % G) == r) ex |= 1ull << (prev_im1 / G);

    uint32_t tk[K];
    bool lane_empty = false;      // no non-excluded local candidate is left
    int npop = 0;                 // entries popped from tk (head is tk[0])
    int hstat = 0;                // head: 0 unknown, 1 absent, 2 visited
    bool pstarted = false;
    uint32_t pbucket = 0, pslot = 0;   // pslot: first free entry of bucket pbucket
    Key pkey{0, 0, 0};
    bool need_scan = false;
    bool eager = true;            // probe every head in the next round
    bool done = !active;
    uint32_t win = kKeyMax;

    issue_priority<kPrioScanEarly, kPrio>();
    // (0) main scan, on as few planes as the wave's current c values allow.
#pragma unroll
    for (int q = 0; q < K; ++q) tk[q] = kKeyMax;
    const int bp = wave_plane_cap<NW>(Pl, active);
    if (active) {
      ncap4 += bp == 4 ? 1u : 0u;
      ncap5 += bp == 5 ? 1u : 0u;
      ncap6 += bp == 6 ? 1u : 0u;
      ncap0 += bp == 0 ? 1u : 0u;
    }
#pragma unroll 1
    for (int sr = 0; sr < nruns; ++sr) {
      const uint32_t e0 = __builtin_amdgcn_readfirstlane(runs[sr]);
      scan_run_priority<kPrio>(sr, nruns);
      const int ib = (int)(e0 >> 8);
      const int ie = (int)(__builtin_amdgcn_readfirstlane(runs[sr + 1]) >> 8);
      with_words<NW, Codes>((int)(e0 & 0xFFu), [&](auto Fc, auto Bc) __attribute__((always_inline)) {
        constexpr int F = decltype(Fc)::value, B = decltype(Bc)::value;
        auto scan = [&](auto BPc) __attribute__((always_inline)) {
          constexpr int BPv = decltype(BPc)::value;
#pragma unroll 1
          for (int it = ib; it < ie; ++it) {
            // i > L reads a dead row whose key ~0 leaves the top-K unchanged
            const int i = r + 1 + G * it;
            topk_insert<K>(tk, eval_key<NW, F, B, BPv>(desc + (i - 1) * Gm::DESC, cols, colbase, Pl,
                                                       sign_of(it), ev));
          }
        };
        if (bp == 4) scan(std::integral_constant<int, 4>{});
        else if (bp == 5) scan(std::integral_constant<int, 5>{});
        else if (bp == 6) scan(std::integral_constant<int, 6>{});
        else scan(std::integral_constant<int, 0>{});
      });
    }
    issue_priority<kPrioResolve, kPrio>();
    // The predecessor is visited: drop it from its owner's top-K.
    if (prev_im1 != 0xFFFFFFFFu && (int)(prev_im1 % G) == r) {
      bool found = false;
#pragma unroll
      for (int q = 0; q < K; ++q) {
        found = found || (tk[q] != kKeyMax && (tk[q] & 0xFFu) == prev_im1);
        if (found) tk[q] = (q + 1 < K) ? tk[q + 1 < K ? q + 1 : q] : kKeyMax;
      }
      // Counts as a pop: after K removals the lane must rescan, while an
      // empty head before that means every local candidate was examined.
      npop = found ? 1 : 0;
    }
    lane_empty = tk[0] == kKeyMax;

    for (;;) {
      // (1) rescan of local candidates, skipping excluded ones (a lane whose
      //     top-K entries were all found visited).
      if (__ballot(!done && need_scan) != 0ull) {
        if (!done && need_scan) {
#pragma unroll
          for (int q = 0; q < K; ++q) tk[q] = kKeyMax;
        }
        const bool scanning = !done && need_scan;
#pragma unroll 1
        for (int sr = 0; sr < nruns; ++sr) {
          const uint32_t e0 = __builtin_amdgcn_readfirstlane(runs[sr]);
          const int ib = (int)(e0 >> 8);
          const int ie = (int)(__builtin_amdgcn_readfirstlane(runs[sr + 1]) >> 8);
          with_words<NW, Codes>((int)(e0 & 0xFFu), [&](auto Fc, auto Bc) __attribute__((always_inline)) {
            constexpr int F = decltype(Fc)::value, B = decltype(Bc)::value;
            uint64_t xw = ex >> ib;
#pragma unroll 1
            for (int it = ib; it < ie; ++it) {
              const bool live = scanning && it < ncand;
              const int i = r + 1 + G * it;              // i > L: dead row
              uint32_t key = eval_key<NW, F, B, 0>(desc + (i - 1) * Gm::DESC, cols, colbase, Pl,
                                                   sign_of(it), ev);
              key |= 0u - (uint32_t)(xw & 1ull);
              xw >>= 1;
              if (live) topk_insert<K>(tk, key);
            }
          });
        }
        if (!done && need_scan) {
          need_scan = false;
          npop = 0;
          hstat = 0;
          pstarted = false;
          eager = true;
          lane_empty = tk[0] == kKeyMax;
        }
      }
      // (2) heads: in a step's first round (and after a rescan) every lane
      //     probes its head at once; later rounds merge the heads by their
      //     known status first and probe only the owner of the group's best
      //     head when its status is still unknown.
      const uint32_t head = tk[0];
      const bool head_valid = !done && !lane_empty && npop < K && head != kKeyMax;
      auto probe_head = [&](uint32_t hk) {
        if (!pstarted) {
          pkey = flip_key_n<KWM>(P, hk & 0xFFu);
          pbucket = bucket_of_hash(hP ^ zob[hk & 0xFFu], a.n_buckets);
          pstarted = true;
        }
        uint32_t fs = 0;
        const int res = scan_bucket<kFLO, kFHI>(table + (uint64_t)pbucket * kBucketBytes, pkey, efmt, fs);
        if (res == 2) {
          hstat = 2;
        } else if (res == 1) {
          hstat = 1;
          pslot = fs;
        } else {
          pbucket = (pbucket + 1u == a.n_buckets) ? 0u : pbucket + 1u;
        }
      };
      issue_priority<kPrioProbe, kPrio>();
      if (head_valid && hstat == 0 && eager) probe_head(head);
      issue_priority<kPrioResolve, kPrio>();
      eager = false;
      // Every head already known to be visited leaves its list now (a visited
      // neighbour is never chosen), so the merge sees only heads that are new
      // or not yet probed: a walk needs another round only when the group's
      // best remaining head has not been probed.
      if (head_valid && hstat == 2) {
        ex |= 1ull << ((head & 0xFFu) / G);
#pragma unroll
        for (int q = 0; q + 1 < K; ++q) tk[q] = tk[q + 1];
        tk[K - 1] = kKeyMax;
        ++npop;
        hstat = 0;
        pstarted = false;
      }
      const uint32_t cur = tk[0];
      const bool cur_valid = !done && !lane_empty && npop < K && cur != kKeyMax;
      // (3) merge the heads of the group.
      const uint32_t my = cur_valid ? cur : kKeyMax;
      const uint32_t gmin = group_min<G>(my);
      const bool owner = cur_valid && my == gmin;
      if (__ballot(owner && hstat == 0) != 0ull) {
        issue_priority<kPrioProbe, kPrio>();
        if (owner && hstat == 0) probe_head(cur);
        issue_priority<kPrioResolve, kPrio>();
      }
      const uint32_t ostat = group_max<G>(owner ? (uint32_t)(hstat + 1) : 0u);
      const bool exhausted_any = group_max<G>((!done && !lane_empty && npop >= K) ? 1u : 0u) != 0u;
      if (!done) {
        if (exhausted_any) {
          // some lane must refill its top-K before the group can decide
        } else if (gmin == kKeyMax) {
          done = true;          // trapped: every neighbour has been visited
          win = kKeyMax;
        } else if (ostat == 2u) {
          done = true;          // the group's best remaining candidate is new
          win = gmin;
        } else if (ostat == 3u) {
          if (owner) {
            ex |= 1ull << ((cur & 0xFFu) / G);
#pragma unroll
            for (int q = 0; q + 1 < K; ++q) tk[q] = tk[q + 1];
            tk[K - 1] = kKeyMax;
            ++npop;
            hstat = 0;
            pstarted = false;
          }
        }
        if (!done && npop >= K && !lane_empty) need_scan = true;
      }
      if (__ballot(!done) == 0ull) break;
    }

    // ---- move ---------------------------------------------------------------
    issue_priority<kPrioMove, kPrio>();
    if (active) {
      if (win == kKeyMax) {
        active = false;         // trapped walk stops here
        trapped = true;
      } else {
        const uint32_t im1 = win & 0xFFu;
        const int32_t dE = 4 * ((int32_t)(win >> 8) - kBias);
        const uint32_t sw = colw[(im1 >> 5) * kBlock + tid];
        apply_move_planes<NW>(desc + im1 * Gm::DESC, cols, colbase, (sw >> (im1 & 31)) & 1u, Pl);
        // negate s_i in both arrays
        colw[(im1 >> 5) * kBlock + tid] = sw ^ (1u << (im1 & 31));
        {
          const int y = L - 1 - (int)im1;
          colw[(Gm::NWA + (y >> 5)) * kBlock + tid] ^= 1u << (y & 31);
        }
        const Key NP = flip_key_n<KWM>(P, im1);
        // the lane that probed the winner inserts it at the slot it found
        const bool owner = hstat == 1 && !lane_empty && npop < K && tk[0] == win;
        if (owner) store_entry<kFLO, kFHI>(table + (uint64_t)pbucket * kBucketBytes, pslot, NP, efmt);
        P = NP;
        hP ^= zob[im1];
        if ((int)(im1 & (uint32_t)(G - 1)) == r) {
          const int li = (int)(im1 >> lgG);
          static_for<0, Gm::kSW>([&](auto wc) {
            constexpr int w = decltype(wc)::value;
            if ((li >> 5) == w) smk[w] ^= 1u << (li & 31);
          });
        }
        E += dE;
        if (E < bestE) { bestE = E; bestP = P; }
        h = mix64(h ^ (((uint64_t)(im1 + 1u) << 32) | (uint64_t)(uint32_t)E));
        if (tracing && r == 0) {
          a.trace_j[walk * a.walk_len + steps] = (int16_t)(im1 + 1u);
          a.trace_E[walk * a.walk_len + steps] = E;
        }
        prev_im1 = im1;
        ++steps;
      }
    }
  }

  const bool finished = trapped || steps >= a.walk_len;
  if (kSv && a.state && slot < n_block && r == 0 && !skip) {
    WalkState o{};
    o.P[0] = P.w0; o.P[1] = P.w1; o.P[2] = P.w2; o.P[3] = P.w3;
    o.bestP[0] = bestP.w0; o.bestP[1] = bestP.w1; o.bestP[2] = bestP.w2; o.bestP[3] = bestP.w3;
    o.h = h;
    o.steps = steps;
    o.bestE = bestE;
    o.prev_jm1 = prev_im1;
    o.trapped = trapped ? 1u : 0u;
    a.state[walk] = o;
  }
  if (kSv && a.wstat && slot < n_block && r == 0 && !skip) a.wstat[walk] = finished ? 2u : 1u;
  if (a.cap_steps && slot < n_block && r == 0 && !skip) {
    uint4 v;
    v.x = ncap4; v.y = ncap5; v.z = ncap6; v.w = ncap0;
    *reinterpret_cast<uint4 *>(a.cap_steps + (uint64_t)walk * 4u) = v;
  }
  if (slot < n_block && r == 0 && !skip && (!kSv || finished)) {
    a.best_seq[walk * KW] = bestP.w0;
    if (KW > 1) a.best_seq[walk * KW + 1] = bestP.w1;
    if (KW > 2) a.best_seq[walk * KW + 2] = bestP.w2;
    if (KW > 3) a.best_seq[walk * KW + 3] = bestP.w3;
    a.best_E[walk] = bestE;
    a.steps_done[walk] = steps;
    if (a.digest) a.digest[walk] = mix64(h ^ (uint64_t)steps);
  }
  if (kSv && a.done_flag) {
    const int all = __syncthreads_and((slot >= n_block || skip || finished) ? 1 : 0);
    if (threadIdx.x == 0 && all) __hip_atomic_store(a.done_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

template <int NW>
__global__ void __launch_bounds__(kBlock, FullOccupancy<NW>::value) full_walk_kernel(const WalkLaunch w) {
  extern __shared__ __align__(16) uint8_t lds[];
  const int64_t first = (int64_t)blockIdx.x * (kBlock / kG);
  FullTask t;
  t.starts = w.starts;
  t.seed = w.seed;
  t.L = w.L;
  t.n_block = (int32_t)min((int64_t)(kBlock / kG), w.n_walks - first);
  t.walk_begin = w.walk_begin + first;
  t.walk_len = w.walk_len;
  t.best_seq = w.best_seq;
  t.best_E = w.best_E;
  t.steps_done = w.steps_done;
  t.digest = w.digest;
  t.trace_j = w.trace_j;
  t.trace_E = w.trace_E;
  t.n_trace = w.n_trace;
  t.cap_steps = w.cap_steps;
  t.tables = w.tables + (uint64_t)first * w.table_bytes;
  t.table_bytes = w.table_bytes;
  t.n_buckets = w.n_buckets;
  t.state = nullptr;
  t.wstat = nullptr;
  t.step_end = w.walk_len;
  t.preempt = nullptr;
  t.done_flag = nullptr;
  run_full_block<NW, entry_format(32 * (NW - 1) + 2), ClassCodes<NW, NW>, false, full_walk_priority(NW)>(t, lds);
}

// Persistent whole-space batch kernel: every workgroup takes (instance, block)
// items from a device counter until the queue is empty.  Built for the
// largest class NHI of a group of classes [NLO, NHI] of equal occupancy;
// shorter lengths skip the unused lag words.
// Waves per SIMD of the batch kernels: plain batches one fewer than the walk
// kernels of their largest class (the union of several classes' run codes
// needs more registers; at the walk kernels' occupancy it spills); the
// serving forms three, spills and all (the 64..255 whole-space request mix is
// served 4 % faster than at two).
__host__ __device__ constexpr int full_batch_occupancy(int nhi, bool serving) {
  return (nhi <= 4 || serving) ? 3 : 2;
}

template <int NLO, int NHI, bool kSv>
__global__ void __launch_bounds__(kBlock, full_batch_occupancy(NHI, kSv)) full_batch_kernel(const BatchLaunch b) {
  extern __shared__ __align__(16) uint8_t lds[];
  __shared__ int64_t s_item;
  uint8_t *arena = b.arena + (uint64_t)blockIdx.x * b.arena_bytes;
  for (;;) {
    __syncthreads();                       // previous item finished, s_item consumed
    if (threadIdx.x == 0) {
      // no further item once the host has asked the launch to stop
      s_item = (kSv && b.preempt && full_stop_requested(b.preempt)) ? b.n_items
                                                                    : (int64_t)atomicAdd(b.counter, 1u);
    }
    __syncthreads();
    const int64_t it = s_item;
    if (it >= b.n_items) break;            // uniform: every wave leaves together
    const BatchItemDev item = b.items[it];
    const BatchInstanceDev &in = b.inst[item.inst];
    FullTask t;
    t.starts = in.starts;
    t.seed = in.seed;
    t.L = in.L;
    t.n_block = item.n_walks;
    t.walk_begin = item.walk_begin;
    t.walk_len = in.walk_len;
    t.best_seq = in.best_seq;
    t.best_E = in.best_E;
    t.steps_done = in.steps_done;
    t.digest = in.digest;
    t.trace_j = in.trace_j;
    t.trace_E = in.trace_E;
    t.n_trace = in.n_trace;
    t.cap_steps = in.cap_steps;
    t.tables = in.tables ? in.tables + (uint64_t)item.walk_begin * in.table_bytes : arena;
    t.table_bytes = in.table_bytes;
    t.n_buckets = in.n_buckets;
    t.state = in.state;
    t.wstat = in.wstat;
    t.step_end = in.step_end;
    t.preempt = b.preempt;
    t.done_flag = b.item_done ? b.item_done + it : nullptr;
    run_full_block<NHI, entry_format(NLO == 1 ? 3 : 32 * (NLO - 1) + 2), ClassCodes<NLO, NHI>, kSv, kBatchPriority>(t, lds);
  }
}

// Class groups of the batch kernels: classes of equal occupancy share the
// largest one's kernel.
__host__ __device__ constexpr int batch_group_of(int nw) { return nw <= 4 ? 4 : (nw <= 7 ? 7 : 8); }

template <int NLO, int NHI, bool kSv>
static hipError_t launch_batch_g(const BatchLaunch &b, int grid, hipStream_t stream) {
  const size_t lds = Geom<NHI>::lds_bytes();
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(full_batch_kernel<NLO, NHI, kSv>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((full_batch_kernel<NLO, NHI, kSv>), dim3((unsigned)grid), dim3(kBlock), lds, stream, b);
  return hipGetLastError();
}

template <int NLO, int NHI, bool kSv>
static hipError_t blocks_per_cu_g(int *blocks) {
  const void *fn = reinterpret_cast<const void *>(full_batch_kernel<NLO, NHI, kSv>);
  const size_t lds = Geom<NHI>::lds_bytes();
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, fn, kBlock, lds);
}

template <int NW>
static hipError_t launch_nw(const WalkLaunch &w, hipStream_t stream) {
  const size_t lds = Geom<NW>::lds_bytes();
  auto kern = full_walk_kernel<NW>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int64_t per_block = kBlock / kG;
  const int64_t blocks = (w.n_walks + per_block - 1) / per_block;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(kBlock), lds, stream, w);
  return hipGetLastError();
}

}  // namespace full

// The serving form of each group's kernel runs every shorter length too
// (classes from 1 up): a serving launch is one grid on the kernel of the
// largest group present.  Plain batches launch each group on its own kernel.
template <bool kSv>
static hipError_t full_blocks_per_cu_s(int variant, int *blocks) {
  switch (variant) {
    case 4: return full::blocks_per_cu_g<1, 4, kSv>(blocks);
    case 7: return full::blocks_per_cu_g<kSv ? 1 : 5, 7, kSv>(blocks);
    default: return full::blocks_per_cu_g<kSv ? 1 : 8, 8, kSv>(blocks);
  }
}


template <bool kSv>
static hipError_t launch_full_batch_s(const BatchLaunch &b, int variant, int grid, hipStream_t stream) {
  switch (variant) {
    case 4: return full::launch_batch_g<1, 4, kSv>(b, grid, stream);
    case 7: return full::launch_batch_g<kSv ? 1 : 5, 7, kSv>(b, grid, stream);
    default: return full::launch_batch_g<kSv ? 1 : 8, 8, kSv>(b, grid, stream);
  }
}

#ifdef LABS_FULL_SERVING_ONLY
// labs_full_serve.hip: the serving forms, compiled in a translation unit of
// their own (in parallel with this one).
hipError_t full_serving_blocks_per_cu(int variant, int *blocks) {
  return full_blocks_per_cu_s<true>(variant, blocks);
}

hipError_t launch_full_serving(const BatchLaunch &b, int variant, int grid, hipStream_t stream) {
  return launch_full_batch_s<true>(b, variant, grid, stream);
}
#else
// Serving forms (labs_full_serve.hip).
hipError_t full_serving_blocks_per_cu(int variant, int *blocks);
hipError_t launch_full_serving(const BatchLaunch &b, int variant, int grid, hipStream_t stream);

int full_lanes_per_walk() { return full::kG; }

int full_batch_variant(int nw) { return full::batch_group_of(nw); }

hipError_t full_batch_blocks_per_cu(int variant, int *blocks, bool serve) {
  return serve ? full_serving_blocks_per_cu(variant, blocks) : full_blocks_per_cu_s<false>(variant, blocks);
}

hipError_t launch_full_batch(const BatchLaunch &b, int variant, int grid, hipStream_t stream, bool serve) {
  if (grid <= 0) return hipSuccess;
  return serve ? launch_full_serving(b, variant, grid, stream) : launch_full_batch_s<false>(b, variant, grid, stream);
}

size_t full_walk_lds_bytes(int32_t L) {
  switch (full_lag_words_for(L)) {
    case 1: return full::Geom<1>::lds_bytes();
    case 2: return full::Geom<2>::lds_bytes();
    case 3: return full::Geom<3>::lds_bytes();
    case 4: return full::Geom<4>::lds_bytes();
    case 5: return full::Geom<5>::lds_bytes();
    case 6: return full::Geom<6>::lds_bytes();
    case 7: return full::Geom<7>::lds_bytes();
    case 8: return full::Geom<8>::lds_bytes();
    default: return 0;
  }
}

hipError_t launch_full_walks(const WalkLaunch &w, hipStream_t stream) {
  if (w.lanes_per_walk != full::kG) return hipErrorInvalidValue;
  switch (full_lag_words_for(w.L)) {
    case 1: return full::launch_nw<1>(w, stream);
    case 2: return full::launch_nw<2>(w, stream);
    case 3: return full::launch_nw<3>(w, stream);
    case 4: return full::launch_nw<4>(w, stream);
    case 5: return full::launch_nw<5>(w, stream);
    case 6: return full::launch_nw<6>(w, stream);
    case 7: return full::launch_nw<7>(w, stream);
    case 8: return full::launch_nw<8>(w, stream);
    default: return hipErrorInvalidValue;
  }
}
#endif

}  // namespace lsaw
