// labs_kernels.hip -- gfx950 kernels of liblabs.so.
//
// Self-avoiding walks over skew-symmetric binary sequences (Boskovic, Herzog
// & Brest, arXiv 2210.15962, Sec. 3, Eq. 2-4, Alg. 2), scored with an exact
// integer neighbour evaluation written for the CDNA4 vector ALUs.
//
// Notation: L odd, D = (L+1)/2 free bits, m = (L-1)/2 even lags k = 2t+2
// (t = 0..m-1).  On a skew-symmetric sequence every odd-lag C_k is zero, and
// negating free bit j (j < D) flips sequence positions j and L+1-j (j = D
// flips the centre only).  Writing s for the sequence, C_t for the even-lag
// autocorrelations and u_t for the change of C_t divided by 4, the move's
// energy change is
//     dE_j = 8 * sum_t u_t C_t + 16 * sum_t u_t^2,
//     u_t  = -s_j (MF_t s_{j+k} + MB_t s_{j-k}),
// where MF selects forward lags that stay inside the sequence (minus the lag
// k0 = L+1-2j, whose pair (j, L+1-j) keeps its product) and MB the backward
// lags.  (Derived from Eq. 1 and Eq. 2.)
//
// Data layout per walk (replicated in each of the lanes cooperating on it):
//   * sequence: four bit arrays in the lane's LDS column -- odd and even
//     sequence positions, each forwards and reversed, so the forward and
//     backward neighbours of any j are one funnel shift away;
//   * C: two's-complement bit planes of c_t = (C_t - 1)/2 in VGPRs, 32 lags
//     per word; sum_t s_t C_t over a mask M is 2 * sum_M (c_t XOR -f_t) + |M|
//     (f_t = 1 where s_t = -1), i.e. XOR, AND and popcount per plane word;
//   * visited set: exact open-addressing table in HBM keyed on the packed
//     free bits (128-byte buckets, linear probing, no deletions).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>
#include "labs_internal.h"
#include "labs_device.h"

namespace lsaw {

// ---------------------------------------------------------------------------
// Geometry of one lag-word class NW (L with ceil(m/32) == NW)
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int lmax_of(int nw) { return (64 * nw + 1) < kLMax ? (64 * nw + 1) : kLMax; }
// Planes of word w: |c_t| <= (L - 64w - 1)/2 for lags of that word, and
// two's complement with B bits holds [-2^(B-1), 2^(B-1)-1].
__host__ __device__ constexpr int planes_of(int nw, int w) {
  return 1 + clog2((lmax_of(nw) - 64 * w - 1) / 2);
}
__host__ __device__ constexpr int plane_off(int nw, int w) {
  int s = 0;
  for (int i = 0; i < w; ++i) s += planes_of(nw, i);
  return s;
}

// Run table: iterations of the candidate loop grouped into runs of constant
// lag-word counts; slot kRunSlots-1 holds the number of runs.
constexpr int kRunSlots = 32;   // at most 12 runs occur (every class, lanes per walk and L)

template <int NW>
struct Geom {
  static constexpr int NWB = (NW + 1) / 2;           // backward lag words
  static constexpr int NWA = NW + NWB + 1;           // words per bit array
  static constexpr int DMAX = (32 * NW + 1) < 192 ? (32 * NW + 1) : 192;
  // Dwords per row: a multiple of 4 (16-byte row reads) that is 4 (mod 8),
  // so the rows the lanes of one walk group read at once (candidates j, j+1,
  // ..., j+7) start on distinct groups of four banks.
  static constexpr int DESC_FIT = ((9 + NW + 2 * NWB) + 3) & ~3;
  static constexpr int DESC = DESC_FIT % 8 == 0 ? DESC_FIT + 4 : DESC_FIT;
  static constexpr int NPW = plane_off(NW, NW);      // plane words in total
  static constexpr int BMAX = planes_of(NW, 0);
  // Descriptor rows: D real rows plus dead rows up to a multiple of the
  // lanes per walk (<= 8), so every lane of the candidate loop reads a row.
  static constexpr int DROWS = DMAX + 24;
  // The lane columns start on a 256-byte boundary (two-address LDS reads
  // with 256-byte strides need no extra base adjustment).
  static constexpr size_t cols_off() { return ((size_t)DROWS * DESC * 4 + 255) & ~(size_t)255; }
  static constexpr size_t runs_off() { return cols_off() + (size_t)4 * NWA * kBlock * 4; }
  static constexpr size_t zob_off() { return runs_off() + kRunSlots * 4; }
  static constexpr size_t lds_bytes() { return zob_off() + (size_t)DMAX * 4; }
};

// Descriptor row of candidate j (dword offsets).
enum : int {
  DS_FOFF = 0,   // byte offset (within a lane column) of forward source word 0
  DS_FSH = 1,    // funnel shift of the forward vector
  DS_BOFF = 2,
  DS_BSH = 3,
  DS_SOFF = 4,   // byte offset of the word holding s_j
  DS_SPOS = 5,   // bit position of s_j in that word
  DS_KC = 6,     // (((2N - 4|MF & MB| + kBias) << 8) | (j - 1)) + 1; dead rows: 0
  DS_N = 7,      // (N - 2 sum_w 2^(B_w - 1) (|MF_w| + |MB_w|)) << 8, two's complement
  DS_N8 = 8,     // N << 8 (planes-capped evaluation, see eval_key)
  DS_MASKS = 9   // MF[NW], MB[NWB], MFB[NWB]
};

// Column layout: array a (0: odd positions forward, 1: even forward,
// 2: odd reversed, 3: even reversed), word w, lane l -> dword
// ((a*NWA + w) * kBlock + l).  Consecutive lanes hit consecutive banks.
template <int NW>
__device__ __forceinline__ uint32_t col_word_off(int a, int w) {
  return (uint32_t)(((a * Geom<NW>::NWA + w) * kBlock) * 4);
}

template <int NW>
__device__ __forceinline__ void build_descriptors(uint32_t *desc, int L) {
  using Gm = Geom<NW>;
  const int D = (L + 1) / 2, m = (L - 1) / 2;
#pragma unroll 1
  for (int j = 1 + (int)threadIdx.x; j <= D; j += blockDim.x) {
    uint32_t *row = desc + (j - 1) * Gm::DESC;
    const int c = j & 1;                         // class: 1 odd positions, 0 even
    const int n_c = c ? D : m;                   // class size
    const int r = (j - 1) >> 1;                  // index of s_j in its class
    const int afwd = c ? 0 : 1, arev = afwd + 2;
    const int fstart = r + 1, bstart = n_c - r;
    row[DS_FOFF] = col_word_off<NW>(afwd, fstart >> 5);
    row[DS_FSH] = (uint32_t)(fstart & 31);
    row[DS_BOFF] = col_word_off<NW>(arev, bstart >> 5);
    row[DS_BSH] = (uint32_t)(bstart & 31);
    row[DS_SOFF] = col_word_off<NW>(afwd, r >> 5);
    row[DS_SPOS] = (uint32_t)(r & 31);
    const int nF = (j < D) ? n_c - 1 - r : 0;    // forward lags inside [1, L]
    const int nB = r;                            // backward lags inside [1, L]
    const int hole = (j < D) ? D - 1 - j : -1;   // lag index of k0 = L+1-2j
    int cntF = 0, cntB = 0, cntFB = 0, signw = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      uint32_t mf = prefix_mask(nF, w);
      if (hole >= 32 * w && hole < 32 * w + 32) mf &= ~(1u << (hole - 32 * w));
      row[DS_MASKS + w] = mf;
      cntF += __builtin_popcount(mf);
      int nw_bits = __builtin_popcount(mf);
      if (w < Gm::NWB) {
        const uint32_t mb = prefix_mask(nB, w);
        const uint32_t mfb = mb & mf;
        row[DS_MASKS + NW + w] = mb;
        row[DS_MASKS + NW + Gm::NWB + w] = mfb;
        cntB += __builtin_popcount(mb);
        cntFB += __builtin_popcount(mfb);
        nw_bits += __builtin_popcount(mb);
      }
      // the sign plane of word w is counted complemented (see eval_key)
      signw += nw_bits << (planes_of(NW, w) - 1);
    }
    const int N = cntF + cntB;
    row[DS_KC] = (((uint32_t)(2 * N - 4 * cntFB + kBias) << 8) | (uint32_t)(j - 1)) + 1u;
    row[DS_N] = (uint32_t)(N - 2 * signw) << 8;
    row[DS_N8] = (uint32_t)N << 8;
#pragma unroll
    for (int i = DS_MASKS + NW + 2 * Gm::NWB; i < Gm::DESC; ++i) row[i] = 0;
  }
  // Dead rows D+1 .. DROWS: all zero, which gives the key ~0 (never chosen).
  for (int t = (int)threadIdx.x; t < (Gm::DROWS - D) * Gm::DESC; t += blockDim.x) desc[D * Gm::DESC + t] = 0u;
}

// Forward / backward neighbour bit vectors of candidate j, its masks and s_j.
template <int NW>
struct CandVec {
  uint32_t fw[NW];
  uint32_t bw[Geom<NW>::NWB];
  uint32_t mf[NW];
  uint32_t mb[Geom<NW>::NWB];
  uint32_t mfb[Geom<NW>::NWB];
  uint32_t sbit;
};

// Loads candidate j's descriptor row and neighbour vectors.  Only the first
// FW forward and BW backward lag words are formed; the caller guarantees every
// later word has an all-zero mask for this candidate (FW, BW wave-uniform).
template <int NW>
__device__ __forceinline__ void load_candidate(const uint32_t *desc_row, const uint8_t *lds,
                                               uint32_t colbase, CandVec<NW> &cv, int FW, int BW) {
  using Gm = Geom<NW>;
  const uint4 d0 = *reinterpret_cast<const uint4 *>(desc_row);
  const uint4 d1 = *reinterpret_cast<const uint4 *>(desc_row + 4);
  const uint32_t *fsrc = reinterpret_cast<const uint32_t *>(lds + colbase + d0.x);
  const uint32_t *bsrc = reinterpret_cast<const uint32_t *>(lds + colbase + d0.z);
  const uint32_t sw = *reinterpret_cast<const uint32_t *>(lds + colbase + d1.x);
  uint32_t lo = fsrc[0];
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    if (w < FW) {
      cv.mf[w] = desc_row[DS_MASKS + w];
      const uint32_t hi = fsrc[(w + 1) * kBlock];
      cv.fw[w] = funnel(hi, lo, d0.y);
      lo = hi;
    } else {
      cv.mf[w] = 0u;
      cv.fw[w] = 0u;
    }
  }
  uint32_t blo = bsrc[0];
#pragma unroll
  for (int w = 0; w < Gm::NWB; ++w) {
    if (w < BW) {
      cv.mb[w] = desc_row[DS_MASKS + NW + w];
      cv.mfb[w] = desc_row[DS_MASKS + NW + Gm::NWB + w];
      const uint32_t hi = bsrc[(w + 1) * kBlock];
      cv.bw[w] = funnel(hi, blo, d0.w);
      blo = hi;
    } else {
      cv.mb[w] = 0u;
      cv.mfb[w] = 0u;
      cv.bw[w] = 0u;
    }
  }
  cv.sbit = (sw >> d1.y) & 1u;
}

// Candidate key of j: ((dE/8 + kBias) << 8) | (j-1), so unsigned order is
// (dE, j) order.  FW forward and BW backward lag words are evaluated; the
// caller guarantees that candidate j has no lag in any later word (its masks
// there are zero), so those words contribute nothing.
//
// Per plane b of word w the count is popcount((c_b XOR f) AND M); for the
// sign plane (b = B_w - 1) the complement popcount(NOT(c_b XOR f) AND M) =
// |M| - popcount(...) is taken instead, so every plane enters the Horner sum
// with a positive weight and the |M| 2^(B_w - 1) excess is a per-candidate
// constant folded into the descriptor (DS_N).
//
// With BP > 0 every lag word is evaluated on its low BP planes only.  This
// is exact when every c_t of the walk fits in BP bits (two's complement), i.e.
// when the stored planes BP-1 and above of every lag word are copies of plane
// BP-1; the caller checks that for every walk of the wave.  Then plane BP-1
// is the sign plane of every word and enters with weight -2^(BP-1).
template <int NW, int FW, int BW, int BP, bool kMadOpen = true>
__device__ __forceinline__ uint32_t eval_key(const uint32_t *row, const uint8_t *lds,
                                             uint32_t colbase, const uint32_t *P, uint32_t sg) {
  using Gm = Geom<NW>;
  static_assert(FW >= 1 && FW <= NW && BW <= Gm::NWB && BW <= FW, "lag-word counts");
  static_assert(BP == 0 || (BP >= 2 && BP <= planes_of(NW, NW - 1)), "plane cap");
  constexpr int BM = BP > 0 ? BP : Gm::BMAX;
  const uint4 d0 = *reinterpret_cast<const uint4 *>(row);
  const uint4 d1 = *reinterpret_cast<const uint4 *>(row + 4);
  const uint32_t *fsrc = reinterpret_cast<const uint32_t *>(lds + colbase + d0.x);
  const uint32_t *bsrc = reinterpret_cast<const uint32_t *>(lds + colbase + d0.z);
  uint32_t fv[FW];
  uint32_t bv[BW > 0 ? BW : 1];
  {
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
  static_for<0, FW>([&](auto wc) {
    constexpr int w = decltype(wc)::value;
    constexpr int off = plane_off(NW, w);
    constexpr int Bw = BP > 0 ? BP : planes_of(NW, w);
    const uint32_t mf = row[DS_MASKS + w];
#pragma unroll
    for (int b = 0; b < Bw - 1; ++b) cnt[b] = popc_add((P[off + b] ^ fv[w]) & mf, cnt[b]);
    if constexpr (BP > 0)
      cnt[Bw - 1] = popc_add((P[off + Bw - 1] ^ fv[w]) & mf, cnt[Bw - 1]);
    else
      cnt[Bw - 1] = popc_add(~(P[off + Bw - 1] ^ fv[w]) & mf, cnt[Bw - 1]);
    if constexpr (w < BW) {
      const uint32_t mb = row[DS_MASKS + NW + w];
#pragma unroll
      for (int b = 0; b < Bw - 1; ++b) cnt[b] = popc_add((P[off + b] ^ bv[w]) & mb, cnt[b]);
      if constexpr (BP > 0)
        cnt[Bw - 1] = popc_add((P[off + Bw - 1] ^ bv[w]) & mb, cnt[Bw - 1]);
      else
        cnt[Bw - 1] = popc_add(~(P[off + Bw - 1] ^ bv[w]) & mb, cnt[Bw - 1]);
      q = popc_add(~(fv[w] ^ bv[w]) & row[DS_MASKS + NW + Gm::NWB + w], q);   // |MFB| - q
    }
  });
  uint32_t H;
  uint32_t nconst;
  if constexpr (BP > 0 && kMadOpen) {
    // sign plane: weight -2^(BP-1), so the Horner sum opens with
    // cnt[BP-2] - 2 cnt[BP-1]
    H = mad_i24<-2>(cnt[BM - 1], cnt[BM - 2]);
    nconst = row[DS_N8];                         // N << 8
#pragma unroll
    for (int b = BM - 3; b >= 0; --b) H = lshl_add<1>(H, cnt[b]);
  } else if constexpr (BP > 0) {
    // the same as a negation and shift-adds (the batch kernels' register
    // allocation runs faster this way)
    H = 0u - cnt[BM - 1];
    nconst = row[DS_N8];
#pragma unroll
    for (int b = BM - 2; b >= 0; --b) H = lshl_add<1>(H, cnt[b]);
  } else {
    H = cnt[BM - 1];                             // complemented sign planes
    nconst = d1.w;                               // (N - 2 Kc) << 8
#pragma unroll
    for (int b = BM - 2; b >= 0; --b) H = lshl_add<1>(H, cnt[b]);
  }
  const uint32_t t = lshl_add<9>(H, nconst);    // (2 X + N) << 8
  const uint32_t kq = lshl_add<11>(q, d1.z);    // (((kc - 8 q) << 8) | (j - 1)) + 1
  // sg = ~0 when s_j = -1: kq - 1 + t; else kq + ~t = kq - 1 - t.
  return kq + sg + ~(t ^ sg);
}

// Smallest plane cap in {4, 5, 6} valid for every active walk of the wave
// (0: none, use the per-word plane counts).  A cap BP is valid for a lane when
// the planes BP..B_w-1 of every lag word equal plane BP-1.
template <int NW>
__device__ __forceinline__ int wave_plane_cap(const uint32_t *P, bool active) {
  uint32_t d4 = 0u, d5 = 0u, d6 = 0u;   // OR of plane differences at b = 4, 5, >= 6
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

// Lag words some candidate of iteration i (j = G*i + 1 .. G*i + G) needs:
// forward words cover the largest forward range (smallest j of either class),
// backward words the largest backward range (largest j).  Returns FW*8 + BW
// with 1 <= FW <= nw, BW <= FW.
__host__ __device__ constexpr int words_of(int i, int D, int G, int nw) {
  const int m = D - 1;
  const int nwb = (nw + 1) / 2;
  const int jlo = G * i + 1;
  const int jhi = (G * i + G < D) ? G * i + G : D;
  int f = 0;
  for (int j = jlo; j <= jlo + 1 && j < D; ++j) {
    const int nc = (j & 1) ? D : m;
    const int nf = nc - 1 - ((j - 1) >> 1);
    f = nf > f ? nf : f;
  }
  const int b = (jhi - 1) >> 1;
  int bw = (b + 31) >> 5;
  bw = bw < nwb ? bw : nwb;
  int fw = (f + 31) >> 5;
  fw = fw < nw ? fw : nw;
  fw = fw > bw ? fw : bw;
  fw = fw > 1 ? fw : 1;
  return fw * 8 + bw;
}

// Set of (FW, BW) codes the candidate loop of a kernel compiled for lag-word
// class nw can meet: lengths of exactly that class (walk kernel) or of every
// class up to it (batch kernel), for G lanes per walk.
__host__ __device__ constexpr uint64_t words_mask(int nw, int G, bool exact_class) {
  uint64_t mask = 0;
  for (int L = 3; L <= lmax_of(nw); L += 2) {
    const int m = (L - 1) / 2, D = (L + 1) / 2;
    const int cls = (m + 31) / 32;
    if (exact_class ? cls != nw : cls > nw) continue;
    for (int i = 0; i < (D + G - 1) / G; ++i) mask |= 1ull << words_of(i, D, G, nw);
  }
  return mask;
}

template <int NW, int G>
struct WordsMask {
  // walk kernels: lengths of exactly class NW; batch kernels: every class up
  // to NW (classes of equal occupancy share the largest one's kernel), any of
  // 2, 4 or 8 lanes per walk
  static constexpr uint64_t value =
      G > 0 ? words_mask(NW, G, true)
            : (words_mask(NW, 2, false) | words_mask(NW, 4, false) | words_mask(NW, 8, false));
};

// Calls f(FW, BW) as compile-time constants for a wave-uniform code; a code
// outside MASK takes the all-words form, which is valid for every candidate.
// Each instantiation of f has exactly one call site.
template <int NW, uint64_t MASK, class F>
__device__ __forceinline__ void with_words(int code, F &&f) {
  constexpr int kFull = NW * 8 + Geom<NW>::NWB;
  constexpr uint64_t kAll = MASK | (1ull << kFull);
  const int eff = ((kAll >> (code & 63)) & 1ull) != 0 ? code : kFull;
  static_for<8, 64>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    constexpr int fw = c >> 3, bw = c & 7;
    if constexpr (((kAll >> c) & 1ull) != 0 && fw <= NW && bw <= Geom<NW>::NWB && bw <= fw) {
      if (eff == c) f(std::integral_constant<int, fw>{}, std::integral_constant<int, bw>{});
    }
  });
}

// c_t += 2u_t on the bit planes for the move j (u from the pre-move vectors):
// u_t = -s_j * (a_t + b_t), a_t = MF_t ? (f_t ? -1 : 1) : 0, b_t likewise.
template <int NW>
__device__ __forceinline__ void apply_move_planes(const CandVec<NW> &cv, uint32_t *P) {
  using Gm = Geom<NW>;
  // s_j = +1 -> add -w = ~w + 1; s_j = -1 -> add w.
  const uint32_t ms = cv.sbit ? 0u : 0xFFFFFFFFu;
  static_for<0, NW>([&](auto wc) {
    constexpr int w = decltype(wc)::value;
    constexpr int Bw = planes_of(NW, w), off = plane_off(NW, w);
    const uint32_t a0 = cv.mf[w], a1 = cv.fw[w] & cv.mf[w];
    uint32_t b0 = 0u, b1 = 0u;
    if constexpr (w < Gm::NWB) { b0 = cv.mb[w]; b1 = cv.bw[w] & b0; }
    // w = a + b as 3-bit two's complement (bit 2 is the sign).
    const uint32_t w0 = a0 ^ b0, c1 = a0 & b0;
    const uint32_t t1 = a1 ^ b1;
    const uint32_t w1 = t1 ^ c1;
    const uint32_t c2 = (t1 & c1) | (a1 & b1);
    const uint32_t w2 = t1 ^ c2;
    const uint32_t u0 = w0 ^ ms, u1 = w1 ^ ms, u2 = w2 ^ ms;
    uint32_t carry = ms;
#pragma unroll
    for (int b = 1; b < Bw; ++b) {
      const uint32_t x = (b == 1) ? u0 : (b == 2) ? u1 : u2;
      const uint32_t p = P[off + b];
      // truth tables over (p, x, carry) = (0xF0, 0xCC, 0xAA): 0x96 = XOR3, 0xE8 = majority
      const uint32_t c_next = __builtin_amdgcn_bitop3_b32(p, x, carry, 0xE8);
      P[off + b] = __builtin_amdgcn_bitop3_b32(p, x, carry, 0x96);
      carry = c_next;
    }
  });
}

// ---------------------------------------------------------------------------
// Walk kernel
// ---------------------------------------------------------------------------
// One workgroup's share of a walk batch: up to kBlock/G walks of one length L.
struct BlockTask {
  const uint64_t *starts;   // first pivots of the walks' instance, or nullptr
  uint64_t seed;            // seeded starts: SplitMix64 of (seed, walk index)
  int32_t L;
  int32_t n_walks;          // walks of this block (<= kBlock / lanes)
  int32_t lanes;            // lanes per walk (1, 2, 4 or 8)
  int64_t walk_begin;       // index of the block's first walk within its instance
  int64_t walk_len;
  uint64_t *best_seq;
  int32_t *best_E;
  int64_t *steps_done;
  uint64_t *digest;
  int16_t *trace_j;
  int32_t *trace_E;
  int64_t n_trace;
  uint32_t *cap_steps;      // [walk][4] scans per plane cap (4, 5, 6, none), or nullptr
  uint8_t *tables;          // visited table of slot s at tables + s * table_bytes
  uint64_t table_bytes;
  uint32_t n_buckets;
  WalkState *state;         // per-walk progress (indexed by walk) or nullptr
  uint8_t *wstat;           // per-walk status (batches only): 0 not started,
                            // 1 resume from state, 2 finished; nullptr: all start
  int64_t step_end;         // moves after which this launch stops a walk
  const uint32_t *preempt;  // batches: host stop flag polled every 64 moves, or nullptr
  uint32_t *done_flag;      // batches: set to 1 if the block ends with every walk finished
};

// A nonzero stop word from the host (fine-grained memory: read past the
// caches).  One lane of the wave reads it, so a poll is one host-memory read.
__device__ __forceinline__ bool stop_requested(const uint32_t *flag) {
  uint32_t v = 0u;
  if (__lane_id() == 0) v = __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  return __builtin_amdgcn_readfirstlane(v) != 0u;
}

// kSv: the serving form of the batch kernel (per-walk status, walks that
// resume at different move counts, the host stop flag, item completion).
template <int NW, int G, int K, bool kSv = false, bool kPrio = true>
__device__ __forceinline__ void run_block(const BlockTask &a, uint8_t *lds) {
  using Gm = Geom<NW>;
  const int Gl = (G > 0) ? G : a.lanes;        // lanes per walk (wave-uniform)
  uint32_t *desc = reinterpret_cast<uint32_t *>(lds);
  uint8_t *cols = lds + Gm::cols_off();

  const int L = a.L, D = (L + 1) / 2, m = (L - 1) / 2;
  const int KW = (D + 63) / 64;
  build_descriptors<NW>(desc, L);
  uint32_t *runs = reinterpret_cast<uint32_t *>(lds + Gm::runs_off());
  const int nmax = (D + Gl - 1) / Gl;           // candidate-loop iterations
  if (threadIdx.x == 0) {
    // Runs of iterations with equal lag-word counts: (first i << 8) | code,
    // then a sentinel (nmax << 8).  Past kRunSlots - 2 runs the last run takes
    // the all-words form, which serves any candidate.
    // A run also ends where the lanes' sign word changes (every 32
    // iterations), so a run reads one sign word.
    int n = 0, prev = -1;
    for (int i = 0; i < nmax; ++i) {
      const int code = words_of(i, D, Gl, NW);
      if (code == prev && (i & 31) != 0) continue;
      if (n == kRunSlots - 2) {
        runs[n - 1] = (runs[n - 1] & ~0xFFu) | (uint32_t)(NW * 8 + Gm::NWB);
        break;
      }
      runs[n++] = ((uint32_t)i << 8) | (uint32_t)code;
      prev = code;
    }
    runs[n] = (uint32_t)nmax << 8;
    runs[kRunSlots - 1] = (uint32_t)n;
  }
  uint32_t *zob = reinterpret_cast<uint32_t *>(lds + Gm::zob_off());
  for (int j = (int)threadIdx.x; j < D; j += blockDim.x) zob[j] = zobrist_word(j);
  const uint4 z = {0u, 0u, 0u, 0u};
  if (kSv && a.wstat) {
    // Walks resumed from an earlier launch keep their tables: clear only the
    // tables of walks that start now.
    const uint64_t n16 = a.table_bytes / 16u;
    for (int sl = 0; sl < a.n_walks; ++sl) {
      if (a.wstat[a.walk_begin + sl] != 0u) continue;      // uniform
      uint4 *p = reinterpret_cast<uint4 *>(a.tables + (uint64_t)sl * a.table_bytes);
#pragma unroll 4
      for (uint64_t i = threadIdx.x; i < n16; i += kBlock) p[i] = z;
    }
  } else {
    // Clear the visited tables of this block's walks (contiguous, coalesced).
    uint4 *p = reinterpret_cast<uint4 *>(a.tables);
    const uint64_t n16 = (uint64_t)a.n_walks * (a.table_bytes / 16u);
#pragma unroll 4
    for (uint64_t i = threadIdx.x; i < n16; i += kBlock) p[i] = z;
  }
  __syncthreads();

  const int tid = (int)threadIdx.x;
  const int r = tid % Gl;                       // lane rank inside the walk group
  const int slot = tid / Gl;                    // walk slot inside the block
  const int64_t walk = a.walk_begin + slot;
  bool active = slot < a.n_walks;
  // Status of the walk from earlier launches (batches with per-walk status).
  const uint32_t wst = (kSv && a.wstat && active) ? (uint32_t)a.wstat[walk] : 0u;
  const bool fresh = wst == 0u;                 // starts at P_1 in this launch
  const bool skip = wst == 2u;                  // finished earlier: nothing to do
  if (skip) active = false;
  const uint32_t colbase = (uint32_t)tid * 4u;
  uint32_t *colw = reinterpret_cast<uint32_t *>(cols);
  // Visited-table entry format of this length, within the formats the
  // kernel's lengths can meet (walk kernels: one class; batches: every class
  // up to NW).
  constexpr int kFLO = G > 0 ? entry_format(32 * (NW - 1) + 2) : kE12;
  constexpr int kFHI = entry_format(Gm::DMAX);
  const int efmt = entry_format(D);
  constexpr int KWM = (Gm::DMAX + 63) / 64;        // key words any length of the class needs

  // ---- first pivot P_1, or the pivot reached by an earlier launch ----------
  Key P{0, 0, 0};
  WalkState ws{};
  if (active && !fresh) {
    ws = a.state[walk];
    P.w0 = ws.P[0];
    P.w1 = ws.P[1];
    P.w2 = ws.P[2];
  } else if (active) {
    auto start_word = [&](int t) -> uint64_t {
      if (t >= KW) return 0ull;
      uint64_t v;
      if (a.starts) {
        v = a.starts[walk * KW + t];
      } else {
        v = mix64(a.seed + 0x9E3779B97F4A7C15ull * ((uint64_t)walk * (uint64_t)KW + (uint64_t)t + 1u));
      }
      const int bits = D - 64 * t;
      if (bits < 64) v &= ((1ull << bits) - 1ull);
      return v;
    };
    P.w0 = start_word(0);
    P.w1 = start_word(1);
    P.w2 = start_word(2);
  }
  if constexpr (KWM < 3) P.w2 = 0;
  if constexpr (KWM < 2) P.w1 = 0;

  // ---- sequence bit arrays (Eq. 2 expansion) -------------------------------
  for (int i = 0; i < 4 * Gm::NWA; ++i) colw[i * kBlock + tid] = 0u;
  const int n1 = D, n0 = m;
#pragma unroll 1
  for (int i = 1; i <= L; ++i) {
    uint32_t bit;
    if (i <= D) bit = key_bit(P, i - 1);
    else bit = key_bit(P, L - i) ^ (uint32_t)((i - D) & 1);   // s_{D+k} = (-1)^k s_{D-k}
    if (bit) {
      const int c = i & 1, rr = (i - 1) >> 1, nc = c ? n1 : n0;
      const int af = c ? 0 : 1;
      colw[(af * Gm::NWA + (rr >> 5)) * kBlock + tid] |= 1u << (rr & 31);
      const int rv = nc - 1 - rr;
      colw[((af + 2) * Gm::NWA + (rv >> 5)) * kBlock + tid] |= 1u << (rv & 31);
    }
  }

  // ---- C_t (even lags) -> planes of c_t = (C_t - 1)/2, and E(P_1) --------------
  uint32_t Pl[Gm::NPW];
#pragma unroll
  for (int i = 0; i < Gm::NPW; ++i) Pl[i] = 0u;
  int32_t E = 0;
  static_for<0, NW>([&](auto wc) {
    constexpr int w = decltype(wc)::value;
    constexpr int Bw = planes_of(NW, w), off = plane_off(NW, w);
#pragma unroll 1
    for (int tb = 0; tb < 32; ++tb) {
      const int t = 32 * w + tb;
      if (t >= m) break;
      const int sh = t + 1;                    // class distance of lag k = 2t+2
      int mism = 0;
      for (int c = 0; c < 2; ++c) {
        const int nc = c ? n1 : n0, af = c ? 0 : 1;
        const int npairs = nc - sh;
        for (int ww = 0; 32 * ww < npairs; ++ww) {
          const uint32_t x = colw[(af * Gm::NWA + ww) * kBlock + tid];
          const int q = ww + (sh >> 5);
          const uint32_t lo = colw[(af * Gm::NWA + q) * kBlock + tid];
          const uint32_t hi = (q + 1 < Gm::NWA) ? colw[(af * Gm::NWA + q + 1) * kBlock + tid] : 0u;
          const uint32_t y = funnel(hi, lo, (uint32_t)(sh & 31));
          const int rem = npairs - 32 * ww;
          const uint32_t msk = rem >= 32 ? 0xFFFFFFFFu : ((1u << rem) - 1u);
          mism += __builtin_popcount((x ^ y) & msk);
        }
      }
      const int32_t Ct = (L - 2 * t - 2) - 2 * mism;
      E += Ct * Ct;
      const int32_t ct = (Ct - 1) >> 1;
#pragma unroll
      for (int b = 0; b < Bw; ++b) Pl[off + b] |= (uint32_t)((ct >> b) & 1) << tb;
    }
  });

  int32_t bestE = E;
  Key bestP = P;
  uint64_t h = 0;
  int64_t steps = 0;
  uint32_t prev_jm1 = 0xFFFFFFFFu;
  bool trapped = false;
  uint8_t *table = a.tables + (uint64_t)(active ? slot : 0) * a.table_bytes;
  if (active && !fresh) {
    bestE = ws.bestE;
    bestP = Key{ws.bestP[0], KWM >= 2 ? ws.bestP[1] : 0ull, KWM >= 3 ? ws.bestP[2] : 0ull};
    h = ws.h;
    steps = ws.steps;
    prev_jm1 = ws.prev_jm1;
    trapped = ws.trapped != 0u;
    if (trapped) active = false;
  }

  // Hash of the pivot (XOR of the words of its set bits).
  uint32_t hP = 0u;
#pragma unroll 1
  for (int jb = 0; jb < D; ++jb) hP ^= key_bit(P, jb) ? zob[jb] : 0u;

  // Insert P_1 (the table is empty: first entry of its home bucket).
  if (active && fresh && r == 0)
    store_entry<kFLO, kFHI>(table + (uint64_t)bucket_of_hash(hP, a.n_buckets) * kBucketBytes, 0u, P, efmt);

  // Local candidates of lane r: j = r + 1 + Gl*i.
  const int ncand = (D - r + Gl - 1) / Gl;       // may be 0 for r >= D
  const int lgG = Gl == 8 ? 3 : Gl == 4 ? 2 : Gl == 2 ? 1 : 0;
  // Signs of the lane's candidates, bit i <-> s_{r+1+Gl*i} = -1 (0 past D),
  // kept in registers: the scan reads s_j from here, the move toggles it.
  constexpr int kGmin = G > 0 ? G : 2;
  constexpr int kSW = ((Gm::DMAX + kGmin - 1) / kGmin + 31) / 32;
  constexpr int kEXW = ((Gm::DMAX + kGmin - 1) / kGmin + 63) / 64;   // 64-bit exclusion words
  uint32_t smk[kSW];
#pragma unroll
  for (int w = 0; w < kSW; ++w) smk[w] = 0u;
#pragma unroll 1
  for (int i = 0; i < nmax; ++i) {
    const int j = r + 1 + Gl * i;
    const uint32_t bit = j <= D ? key_bit(P, j - 1) : 0u;
    static_for<0, kSW>([&](auto wc) {
      constexpr int w = decltype(wc)::value;
      if ((i >> 5) == w) smk[w] |= bit << (i & 31);
    });
  }
  auto sign_word = [&](int q) -> uint32_t {      // smk[q] for a wave-uniform q
    if constexpr (kSW == 1) {
      return smk[0];
    } else {
      uint32_t wv = 0u;
      static_for<0, kSW>([&](auto wc) {
        constexpr int w = decltype(wc)::value;
        wv |= smk[w] & (0u - (uint32_t)(q == w));
      });
      return wv;
    }
  };
  auto sign_of = [&](int i) -> uint32_t {        // ~0 if s_j = -1, else 0 (i uniform)
    if constexpr (kSW == 1) {
      return (uint32_t)__builtin_amdgcn_sbfe((int)smk[0], i & 31, 1);   // i < 32
    } else {
      // word select with masks (a select chain becomes a stack lookup table)
      uint32_t wv = 0u;
      static_for<0, kSW>([&](auto wc) {
        constexpr int w = decltype(wc)::value;
        wv |= smk[w] & (0u - (uint32_t)((i >> 5) == w));
      });
      return (uint32_t)__builtin_amdgcn_sbfe((int)wv, i & 31, 1);
    }
  };
  const int nruns = (int)__builtin_amdgcn_readfirstlane(runs[kRunSlots - 1]);
  constexpr uint64_t kMask = WordsMask<NW, G>::value;
  // Scans per plane cap are wave-uniform while a walk moves: counted once
  // per wave (scalar registers) and written out for a walk when it stops.
  uint32_t scap4 = 0u, scap5 = 0u, scap6 = 0u, scap0 = 0u;
  auto write_caps = [&]() {
    if (a.cap_steps && slot < a.n_walks && r == 0) {
      uint4 v;
      v.x = scap4; v.y = scap5; v.z = scap6; v.w = scap0;
      *reinterpret_cast<uint4 *>(a.cap_steps + (uint64_t)walk * 4u) = v;
    }
  };
  const bool tracing = active && walk < a.n_trace;

  // Walk kernels and plain batches: every walk starts at move 0, so the step
  // counter is the walks' move count.  Serving: walks resumed from earlier
  // launches may stand at different move counts (a wave can hold walks that
  // ran in different waves before); the wave makes as many moves as its
  // nearest-to-done walk has left, and walks still short of the end are
  // saved unfinished and continue in the next launch.
  const int64_t step_stop = min(a.step_end, a.walk_len);
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
    if (kSv && a.preempt && (step & 63) == 63 && stop_requested(a.preempt)) break;
    // Excluded local candidates (bit i <-> j = r + 1 + Gl*i): the predecessor,
    // then every candidate found visited during this step.
    uint64_t ex0 = 0ull, ex1 = 0ull, ex2 = 0ull;
    auto exclude = [&](uint32_t li) {
      const uint64_t bit = 1ull << (li & 63u);
      if constexpr (kEXW == 1) {
        ex0 |= bit;
      } else {
        const uint32_t q = li >> 6;
        ex0 |= (q == 0u) ? bit : 0ull;
        ex1 |= (q == 1u) ? bit : 0ull;
        if constexpr (kEXW >= 3) ex2 |= (q == 2u) ? bit : 0ull;
      }
    };
    if (prev_jm1 != 0xFFFFFFFFu && (int)(prev_jm1 % Gl) == r) exclude(prev_jm1 / Gl);

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
    // (0) main scan: every local candidate goes into the top-K, evaluated on
    //     as few C planes as the wave's current C values allow.
#pragma unroll
    for (int i = 0; i < K; ++i) tk[i] = kKeyMax;
    const int bp = wave_plane_cap<NW>(Pl, active);
    scap4 += bp == 4 ? 1u : 0u;
    scap5 += bp == 5 ? 1u : 0u;
    scap6 += bp == 6 ? 1u : 0u;
    scap0 += bp == 0 ? 1u : 0u;
#pragma unroll 1
    for (int sr = 0; sr < nruns; ++sr) {
      const uint32_t e0 = __builtin_amdgcn_readfirstlane(runs[sr]);
      scan_run_priority<kPrio>(sr, nruns);
      const int ib = (int)(e0 >> 8);
      const int ie = (int)(__builtin_amdgcn_readfirstlane(runs[sr + 1]) >> 8);
      with_words<NW, kMask>((int)(e0 & 0xFFu), [&](auto Fc, auto Bc) __attribute__((always_inline)) {
        constexpr int F = decltype(Fc)::value, B = decltype(Bc)::value;
        // the run's sign word (runs do not cross a multiple of 32 iterations)
        const uint32_t swr = sign_word(ib >> 5);
        auto scan = [&](auto BPc) __attribute__((always_inline)) {
          constexpr int BPv = decltype(BPc)::value;
#pragma unroll 1
          for (int i = ib; i < ie; ++i) {
            // j > D reads a dead row whose key ~0 leaves the top-K unchanged
            const int j = r + 1 + Gl * i;
            topk_insert<K>(tk, eval_key<NW, F, B, BPv, (G > 0)>(desc + (j - 1) * Gm::DESC, cols, colbase, Pl,
                                                       (uint32_t)__builtin_amdgcn_sbfe((int)swr, i & 31, 1)));
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
    if (prev_jm1 != 0xFFFFFFFFu && (int)(prev_jm1 % Gl) == r) {
      bool found = false;
#pragma unroll
      for (int i = 0; i < K; ++i) {
        found = found || (tk[i] != kKeyMax && (tk[i] & 0xFFu) == prev_jm1);
        if (found) tk[i] = (i + 1 < K) ? tk[i + 1 < K ? i + 1 : i] : kKeyMax;
      }
      // Counts as a pop: after K removals the lane must rescan, while an
      // empty head before that means every local candidate was examined.
      npop = found ? 1 : 0;
    }
    need_scan = false;
    lane_empty = tk[0] == kKeyMax;

    for (;;) {
      // (1) rescan of local candidates, skipping excluded ones (a lane whose
      //     top-K entries were all found visited).
      if (__ballot(!done && need_scan) != 0ull) {
        if (!done && need_scan) {
#pragma unroll
          for (int i = 0; i < K; ++i) tk[i] = kKeyMax;
        }
        const bool scanning = !done && need_scan;
#pragma unroll 1
        for (int sr = 0; sr < nruns; ++sr) {
          const uint32_t e0 = __builtin_amdgcn_readfirstlane(runs[sr]);
          const int ib = (int)(e0 >> 8);
          const int ie = (int)(__builtin_amdgcn_readfirstlane(runs[sr + 1]) >> 8);
          with_words<NW, kMask>((int)(e0 & 0xFFu), [&](auto Fc, auto Bc) __attribute__((always_inline)) {
            constexpr int F = decltype(Fc)::value, B = decltype(Bc)::value;
            // select with masks: a select chain becomes a stack lookup table
            auto ex_word = [&](int qw) {
              if constexpr (kEXW == 1) return ex0;
              else
                return (ex0 & (0ull - (uint64_t)(qw == 0))) | (ex1 & (0ull - (uint64_t)(qw == 1))) |
                       (ex2 & (0ull - (uint64_t)(qw == 2)));
            };
            uint64_t xw = ex_word(ib >> 6) >> (ib & 63);
#pragma unroll 1
            for (int i = ib; i < ie; ++i) {
              if ((i & 63) == 0) xw = ex_word(i >> 6);
              const bool live = scanning && i < ncand;
              const int j = r + 1 + Gl * i;             // j > D: dead row
              uint32_t key = eval_key<NW, F, B, 0>(desc + (j - 1) * Gm::DESC, cols, colbase, Pl, sign_of(i));
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
      // (2) heads.  In a step's first round (and after a lane's rescan) every
      //     lane probes its head at once; later rounds first merge the heads
      //     by their known status and probe only the owner of the group's
      //     best head when that status is still unknown, so a round whose
      //     best head was probed earlier costs no memory access.
      const uint32_t head = tk[0];
      const bool head_valid = !done && !lane_empty && npop < K && head != kKeyMax;
      auto probe_head = [&](uint32_t hk) {
        if (!pstarted) {
          pkey = flip_key_n<KWM>(P, hk & 0xFFu);
          pbucket = bucket_of_hash(hP ^ zob[hk & 0xFFu], a.n_buckets);
          pstarted = true;
        }
        uint32_t slot = 0;
        const int res = scan_bucket<kFLO, kFHI>(table + (uint64_t)pbucket * kBucketBytes, pkey, efmt, slot);
        if (res == 2) {
          hstat = 2;
        } else if (res == 1) {
          hstat = 1;
          pslot = slot;
        } else {
          pbucket = (pbucket + 1u == a.n_buckets) ? 0u : pbucket + 1u;
        }
      };
      // Removes the head (found visited).
      auto pop_head = [&]() {
        exclude((tk[0] & 0xFFu) / Gl);
#pragma unroll
        for (int q = 0; q + 1 < K; ++q) tk[q] = tk[q + 1];
        tk[K - 1] = kKeyMax;
        ++npop;
        hstat = 0;
        pstarted = false;
      };
      issue_priority<kPrioProbe, kPrio>();
      if (head_valid && hstat == 0 && eager) probe_head(head);
      issue_priority<kPrioResolve, kPrio>();
      eager = false;
      // Every head already known to be visited leaves its list now (a visited
      // neighbour is never chosen), so the merge sees only heads that are new
      // or not yet probed: a walk needs another round only when the group's
      // best remaining head has not been probed.
      if (head_valid && hstat == 2) pop_head();
      const uint32_t cur = tk[0];
      const bool cur_valid = !done && !lane_empty && npop < K && cur != kKeyMax;
      // (3) merge the heads of the group.
      const uint32_t my = cur_valid ? cur : kKeyMax;
      const uint32_t gmin = grp_min<G>(my, Gl);
      const bool owner = cur_valid && my == gmin;
      if (__ballot(owner && hstat == 0) != 0ull) {
        issue_priority<kPrioProbe, kPrio>();
        if (owner && hstat == 0) probe_head(cur);
        issue_priority<kPrioResolve, kPrio>();
      }
      const uint32_t ostat = grp_max<G>(owner ? (uint32_t)(hstat + 1) : 0u, Gl);
      const bool exhausted_any = grp_max<G>((!done && !lane_empty && npop >= K) ? 1u : 0u, Gl) != 0u;
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
          if (owner) pop_head();
        }
        if (!done && npop >= K && !lane_empty) need_scan = true;
      }
      if (__ballot(!done) == 0ull) break;
    }

    // ---- move -------------------------------------------------------------
    issue_priority<kPrioMove, kPrio>();
    if (active) {
      if (win == kKeyMax) {
        active = false;         // trapped walk stops here
        trapped = true;
        write_caps();           // the scans this walk took, up to its last
      } else {
        const uint32_t jm1 = win & 0xFFu;
        const int32_t dE = 8 * ((int32_t)(win >> 8) - kBias);
        CandVec<NW> cv;
        load_candidate<NW>(desc + jm1 * Gm::DESC, cols, colbase, cv, NW, Gm::NWB);
        apply_move_planes<NW>(cv, Pl);
        // flip sequence positions j and L+1-j (same class) in all arrays, as
        // LDS xor without return (no read-modify-write round trips; each lane
        // owns its column words)
        const int j = (int)jm1 + 1;
        const int c = j & 1, nc = c ? n1 : n0, af = c ? 0 : 1;
        auto flip = [&](int word, int bit) {
          __hip_atomic_fetch_xor(&colw[word * kBlock + tid], 1u << bit, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WAVEFRONT);
        };
        {
          const int rr = (j - 1) >> 1, rv = nc - 1 - rr;
          flip(af * Gm::NWA + (rr >> 5), rr & 31);
          flip((af + 2) * Gm::NWA + (rv >> 5), rv & 31);
        }
        if (j < D) {
          const int q = L + 1 - j;
          const int rr = (q - 1) >> 1, rv = nc - 1 - rr;
          flip(af * Gm::NWA + (rr >> 5), rr & 31);
          flip((af + 2) * Gm::NWA + (rv >> 5), rv & 31);
        }
        const Key NP = flip_key_n<KWM>(P, jm1);
        // the lane that probed the winner inserts it at the slot it found
        const bool owner = hstat == 1 && !lane_empty && npop < K && tk[0] == win;
        if (owner) store_entry<kFLO, kFHI>(table + (uint64_t)pbucket * kBucketBytes, pslot, NP, efmt);
        P = NP;
        hP ^= zob[jm1];
        if ((int)(jm1 & (uint32_t)(Gl - 1)) == r) {
          const int li = (int)(jm1 >> lgG);
          static_for<0, kSW>([&](auto wc) {
            constexpr int w = decltype(wc)::value;
            if ((li >> 5) == w) smk[w] ^= 1u << (li & 31);
          });
        }
        E += dE;
        if (E < bestE) { bestE = E; bestP = P; }
        h = mix64(h ^ (((uint64_t)(jm1 + 1u) << 32) | (uint64_t)(uint32_t)E));
        if (tracing && r == 0) {
          a.trace_j[walk * a.walk_len + steps] = (int16_t)(jm1 + 1u);
          a.trace_E[walk * a.walk_len + steps] = E;
        }
        prev_jm1 = jm1;
        ++steps;
      }
    }
  }

  const bool finished = trapped || steps >= a.walk_len;
  if (a.state && slot < a.n_walks && r == 0 && !skip) {
    WalkState o{};
    o.P[0] = P.w0; o.P[1] = P.w1; o.P[2] = P.w2;
    o.bestP[0] = bestP.w0; o.bestP[1] = bestP.w1; o.bestP[2] = bestP.w2;
    o.h = h;
    o.steps = steps;
    o.bestE = bestE;
    o.prev_jm1 = prev_jm1;
    o.trapped = trapped ? 1u : 0u;
    a.state[walk] = o;
  }
  if (kSv && a.wstat && slot < a.n_walks && r == 0 && !skip) a.wstat[walk] = finished ? 2u : 1u;
  if (!trapped && !skip) write_caps();   // moved at every step of this launch
  if (finished && slot < a.n_walks && r == 0 && !skip) {
    a.best_seq[walk * KW] = bestP.w0;
    if (KW > 1) a.best_seq[walk * KW + 1] = bestP.w1;
    if (KW > 2) a.best_seq[walk * KW + 2] = bestP.w2;
    a.best_E[walk] = bestE;
    a.steps_done[walk] = steps;
    if (a.digest) a.digest[walk] = mix64(h ^ (uint64_t)steps);
  }
  if (kSv && a.done_flag) {
    const int all = __syncthreads_and((slot >= a.n_walks || skip || finished) ? 1 : 0);
    if (threadIdx.x == 0 && all) __hip_atomic_store(a.done_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

template <int NW, int G, int K>
__global__ void __launch_bounds__(kBlock) walk_kernel(const WalkLaunch w) {
  extern __shared__ __align__(16) uint8_t lds[];
  const int64_t first = (int64_t)blockIdx.x * (kBlock / G);
  BlockTask t;
  t.starts = w.starts;
  t.seed = w.seed;
  t.L = w.L;
  t.n_walks = (int32_t)min((int64_t)(kBlock / G), w.n_walks - first);
  t.lanes = G;
  t.walk_begin = w.walk_begin + first;
  t.walk_len = w.walk_len;
  t.best_seq = w.best_seq;
  t.best_E = w.best_E;
  t.steps_done = w.steps_done;
  t.digest = w.digest;
  t.trace_j = w.trace_j;
  t.trace_E = w.trace_E;
  t.n_trace = w.n_trace;
  t.tables = w.tables + (uint64_t)first * w.table_bytes;
  t.table_bytes = w.table_bytes;
  t.n_buckets = w.n_buckets;
  t.cap_steps = w.cap_steps;
  t.state = nullptr;
  t.wstat = nullptr;
  t.step_end = w.walk_len;
  t.preempt = nullptr;
  t.done_flag = nullptr;
  run_block<NW, G, K, false, walk_priority(NW)>(t, lds);
}

// ---------------------------------------------------------------------------
// Persistent mixed-length batch kernel: every workgroup takes (instance, block)
// items from a device counter until the queue is empty, running each item with
// the variant compiled for its lag-word class and lanes per walk.
// ---------------------------------------------------------------------------

// Waves per SIMD the batch kernel of a class is built for: three (168 VGPRs)
// up to class 5 -- class 5 spills a few dwords there, and still runs the
// 121..301 request mix 6 % faster than at two waves -- and two for class 6.
template <int NWMAX>
struct BatchOccupancy { static constexpr int value = NWMAX <= 5 ? 3 : 2; };

template <int NWMAX, bool kSv>
__global__ void __launch_bounds__(kBlock, BatchOccupancy<NWMAX>::value) batch_kernel(const BatchLaunch b) {
  extern __shared__ __align__(16) uint8_t lds[];
  __shared__ int64_t s_item;
  uint8_t *arena = b.arena + (uint64_t)blockIdx.x * b.arena_bytes;
  for (;;) {
    __syncthreads();                       // previous item finished, s_item consumed
    if (threadIdx.x == 0) {
      // no further item once the host has asked the launch to stop
      s_item = (kSv && b.preempt && stop_requested(b.preempt)) ? b.n_items : (int64_t)atomicAdd(b.counter, 1u);
    }
    __syncthreads();
    const int64_t it = s_item;
    if (it >= b.n_items) break;            // uniform: every wave leaves together
    const BatchItemDev item = b.items[it];
    const BatchInstanceDev &in = b.inst[item.inst];
    BlockTask t;
    t.starts = in.starts;
    t.seed = in.seed;
    t.L = in.L;
    t.n_walks = item.n_walks;
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
    t.lanes = item.code & 15;
    // Compiled for the largest lag-word class of the batch: shorter lengths
    // skip the unused lag words (uniform guards), lanes per walk is a runtime
    // value, so one code path serves every item.
    run_block<NWMAX, 0, 3, kSv, kBatchPriority>(t, lds);
  }
}

__global__ void batch_reset_kernel(uint32_t *counter) {
  if (threadIdx.x == 0) *counter = 0u;
}

// ---------------------------------------------------------------------------
// Energy of full sequences (Eq. 1): one wavefront per sequence, bits in LDS.
// ---------------------------------------------------------------------------
constexpr int kEnergyWaves = 4;
constexpr int kEnergyWords = kEnergyLMax / 32 + 2;

__global__ void __launch_bounds__(64 * kEnergyWaves) energy_kernel(const int8_t *seqs, int32_t L,
                                                                 int64_t n, int32_t *E_out) {
  __shared__ uint32_t bits[kEnergyWaves][kEnergyWords];
  const int wave = (int)threadIdx.x / 64, lane = (int)threadIdx.x % 64;
  const int nw = (L + 31) / 32;
  for (int64_t seq = (int64_t)blockIdx.x * kEnergyWaves + wave; seq < n;
       seq += (int64_t)gridDim.x * kEnergyWaves) {
    const int8_t *s = seqs + seq * (int64_t)L;
    for (int base = 0; base < L; base += 64) {
      const int i = base + lane;
      const bool neg = i < L && s[i] < 0;
      const uint64_t bal = __ballot(neg);
      if (lane == 0) {
        bits[wave][base / 32] = (uint32_t)bal;
        if (base / 32 + 1 < kEnergyWords) bits[wave][base / 32 + 1] = (uint32_t)(bal >> 32);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    int64_t acc = 0;
    for (int k = 1 + lane; k < L; k += 64) {
      const int npairs = L - k, q = k >> 5, sh = k & 31;
      int mism = 0;
      for (int w = 0; 32 * w < npairs; ++w) {
        const uint32_t x = bits[wave][w];
        const uint32_t lo = bits[wave][w + q];
        const uint32_t hi = (w + q + 1 < kEnergyWords) ? bits[wave][w + q + 1] : 0u;
        const uint32_t y = funnel(hi, lo, (uint32_t)sh);
        const int rem = npairs - 32 * w;
        const uint32_t msk = rem >= 32 ? 0xFFFFFFFFu : ((1u << rem) - 1u);
        mism += __builtin_popcount((x ^ y) & msk);
      }
      const int64_t Ck = (int64_t)npairs - 2 * mism;
      acc += Ck * Ck;
    }
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) E_out[seq] = (int32_t)acc;
    __builtin_amdgcn_wave_barrier();
  }
}

__global__ void starts_kernel(int32_t L, int64_t n_walks, uint64_t seed, uint64_t *out) {
  const int D = (L + 1) / 2, KW = (D + 63) / 64;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n_walks * KW;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t w = idx / KW;
    const int t = (int)(idx % KW);
    uint64_t v = mix64(seed + 0x9E3779B97F4A7C15ull * ((uint64_t)w * (uint64_t)KW + (uint64_t)t + 1u));
    const int bits = D - 64 * t;
    if (bits < 64) v &= ((1ull << bits) - 1ull);
    out[idx] = v;
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_energy(const int8_t *seqs, int32_t L, int64_t n, int32_t *E_out,
                         hipStream_t stream) {
  if (n == 0) return hipSuccess;
  int64_t blocks = (n + kEnergyWaves - 1) / kEnergyWaves;
  if (blocks > 65535) blocks = 65535;
  hipLaunchKernelGGL(energy_kernel, dim3((unsigned)blocks), dim3(64 * kEnergyWaves), 0, stream,
                     seqs, L, n, E_out);
  return hipGetLastError();
}

hipError_t launch_starts(int32_t L, int64_t n_walks, uint64_t seed, uint64_t *out,
                         hipStream_t stream) {
  if (n_walks == 0) return hipSuccess;
  const int KW = key_words_for(L);
  int64_t blocks = (n_walks * KW + 255) / 256;
  if (blocks > 65535) blocks = 65535;
  hipLaunchKernelGGL(starts_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, L, n_walks, seed, out);
  return hipGetLastError();
}

template <int NW>
static size_t lds_for() { return Geom<NW>::lds_bytes(); }

size_t walk_lds_bytes(int32_t L) {
  switch (lag_words_for(L)) {
    case 1: return lds_for<1>();
    case 2: return lds_for<2>();
    case 3: return lds_for<3>();
    case 4: return lds_for<4>();
    case 5: return lds_for<5>();
    case 6: return lds_for<6>();
    default: return 0;
  }
}

template <int NW, int G>
static hipError_t launch_nw_g(const WalkLaunch &w, hipStream_t stream) {
  constexpr int K = (G == 1) ? 4 : 3;
  const size_t lds = Geom<NW>::lds_bytes();
  auto kern = walk_kernel<NW, G, K>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int64_t per_block = kBlock / G;
  const int64_t blocks = (w.n_walks + per_block - 1) / per_block;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(kBlock), lds, stream, w);
  return hipGetLastError();
}

template <int NW>
static hipError_t launch_nw(const WalkLaunch &w, hipStream_t stream) {
  switch (w.lanes_per_walk) {
    case 1: return launch_nw_g<NW, 1>(w, stream);
    case 2: return launch_nw_g<NW, 2>(w, stream);
    case 4: return launch_nw_g<NW, 4>(w, stream);
    case 8: return launch_nw_g<NW, 8>(w, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_walks(const WalkLaunch &w, hipStream_t stream) {
  switch (lag_words_for(w.L)) {
    case 1: return launch_nw<1>(w, stream);
    case 2: return launch_nw<2>(w, stream);
    case 3: return launch_nw<3>(w, stream);
    case 4: return launch_nw<4>(w, stream);
    case 5: return launch_nw<5>(w, stream);
    case 6: return launch_nw<6>(w, stream);
    default: return hipErrorInvalidValue;
  }
}


// One batch kernel per lag-word class (NW 1 and 2 share the first), so that
// each class runs at the occupancy of its own register footprint.
int batch_variant(int nw) { return nw <= 2 ? 2 : (nw > 6 ? 6 : nw); }

size_t batch_lds_bytes(int variant) {
  switch (variant) {
    case 2: return lds_for<2>();
    case 3: return lds_for<3>();
    case 4: return lds_for<4>();
    case 5: return lds_for<5>();
    default: return lds_for<6>();
  }
}

template <int V>
static const void *batch_fn(bool serve) {
  return serve ? reinterpret_cast<const void *>(batch_kernel<V, true>)
               : reinterpret_cast<const void *>(batch_kernel<V, false>);
}

static const void *batch_kernel_ptr(int variant, bool serve) {
  switch (variant) {
    case 2: return batch_fn<2>(serve);
    case 3: return batch_fn<3>(serve);
    case 4: return batch_fn<4>(serve);
    case 5: return batch_fn<5>(serve);
    default: return batch_fn<6>(serve);
  }
}

hipError_t batch_blocks_per_cu(int variant, int *blocks, bool serve) {
  const void *fn = batch_kernel_ptr(variant, serve);
  const size_t lds = batch_lds_bytes(variant);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, fn, kBlock, lds);
}

hipError_t launch_batch_reset(uint32_t *counter, hipStream_t stream) {
  hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, stream, counter);
  return hipGetLastError();
}

template <int V, bool kSv>
static hipError_t launch_batch_v(const BatchLaunch &b, int grid, hipStream_t stream) {
  const size_t lds = Geom<V>::lds_bytes();
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(batch_kernel<V, kSv>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((batch_kernel<V, kSv>), dim3((unsigned)grid), dim3(kBlock), lds, stream, b);
  return hipGetLastError();
}

template <bool kSv>
static hipError_t launch_batch_s(const BatchLaunch &b, int variant, int grid, hipStream_t stream) {
  switch (variant) {
    case 2: return launch_batch_v<2, kSv>(b, grid, stream);
    case 3: return launch_batch_v<3, kSv>(b, grid, stream);
    case 4: return launch_batch_v<4, kSv>(b, grid, stream);
    case 5: return launch_batch_v<5, kSv>(b, grid, stream);
    default: return launch_batch_v<6, kSv>(b, grid, stream);
  }
}

hipError_t launch_batch(const BatchLaunch &b, int variant, int grid, hipStream_t stream, bool serve) {
  if (grid <= 0) return hipSuccess;
  return serve ? launch_batch_s<true>(b, variant, grid, stream) : launch_batch_s<false>(b, variant, grid, stream);
}

}  // namespace lsaw
