// labs_oracle.cpp -- TEST INFRASTRUCTURE ONLY.
//
// Plain, slow, obviously-correct CPU reference ("oracle") for the
// skew-symmetric LABS self-avoiding walk of Boskovic, Herzog & Brest,
// "Parallel Self-Avoiding Walks for a Low-Autocorrelation Binary Sequences
// Problem" (arXiv 2210.15962).  Only the tests, the smoke check and the CPU
// baseline leg of the benchmark may load this library.  It shares no code,
// header, table or helper with the GPU library; it never uses the
// incremental neighbour evaluation: every energy is recomputed from Eq. 1.
//
// Conventions (the walk and its packing):
//   * L odd, 3 <= L <= ORC_L_MAX; D = (L+1)/2 free bits x_1..x_D (Eq. 2).
//   * Packed key: W = ceil(D/64) uint64 words; free bit x_j is bit (j-1)%64
//     of word (j-1)/64; bit value 1 means -1; unused high bits are zero.
//   * A neighbour of a pivot negates one free bit (Sec. 3: D neighbours).
//   * walk_len is the number of moves (Alg. 2 creates P_2..P_{n+1}).
//   * Next pivot = the unvisited neighbour of lowest energy, ties broken to
//     the lowest j (Eq. 3 with a lowest-index tie rule).
//   * If every neighbour has been visited the walk stops early.
//   * Best tracking uses strict "<" starting from E(P_1) (Alg. 2).
//   * Digest: h = mix64(h ^ (j<<32 | (uint32)E)) per move, final
//     mix64(h ^ steps).  mix64 is the SplitMix64 finaliser (Steele, Lea &
//     Flood, OOPSLA 2014).
//   * Random starts: word t of walk w = mix64(seed + G*(w*W + t + 1)) with
//     G = 0x9E3779B97F4A7C15, masked to the D valid bits.
//
// The whole search space (the sokol_full solver that Sec. 5 names as future
// work) uses the same walk rules on all 2^L sequences of any length L: the
// state is the whole sequence (L bits packed like a key, bit i-1 = s_i,
// 1 means -1), a neighbour negates one sequence position (L neighbours), and
// starts draw W = ceil(L/64) words masked to L bits.
#include <cstdint>
#include <cstring>
#include <set>
#include <array>
#include <vector>
#include <thread>
#include <atomic>

namespace {

constexpr int ORC_L_MAX = 383;           // D <= 192, so W <= 3
constexpr int ORC_W_MAX = 4;
constexpr int ORC_FULL_L_MAX = 255;      // whole space: L bits, W <= 4

typedef std::array<uint64_t, ORC_W_MAX> Key;

int free_bits(int L) { return (L + 1) / 2; }
int key_words(int D) { return (D + 63) / 64; }
bool valid_skew_L(int L) { return L >= 3 && L <= ORC_L_MAX && (L % 2) == 1; }
bool valid_full_L(int L) { return L >= 3 && L <= ORC_FULL_L_MAX; }

// Eq. 1: C_k = sum_{i=1}^{L-k} s_i s_{i+k};  E = sum_{k=1}^{L-1} C_k^2.
int64_t energy_direct(const int8_t* s, int L) {
  int64_t E = 0;
  for (int k = 1; k <= L - 1; ++k) {
    int64_t c = 0;
    for (int i = 0; i + k < L; ++i) c += (int64_t)s[i] * (int64_t)s[i + k];
    E += c * c;
  }
  return E;
}

// Eq. 2: s_j = x_j for j <= D; s_{D+i} = (-1)^i s_{D-i}, i = 1..D-1.
void expand_skew(const int8_t* x, int L, int8_t* s) {
  int D = free_bits(L);
  for (int j = 1; j <= D; ++j) s[j - 1] = x[j - 1];
  for (int i = 1; i <= D - 1; ++i) {
    int8_t v = s[D - i - 1];
    s[D + i - 1] = (i % 2 == 0) ? v : (int8_t)(-v);
  }
}

void unpack_key(const uint64_t* key, int D, int8_t* x) {
  for (int j = 1; j <= D; ++j) {
    uint64_t bit = (key[(j - 1) / 64] >> ((j - 1) % 64)) & 1u;
    x[j - 1] = bit ? (int8_t)-1 : (int8_t)1;
  }
}

Key pack_key(const int8_t* x, int D) {
  Key k{};
  for (int j = 1; j <= D; ++j)
    if (x[j - 1] < 0) k[(j - 1) / 64] |= (uint64_t)1 << ((j - 1) % 64);
  return k;
}

int64_t energy_of_free_bits(const int8_t* x, int L, std::vector<int8_t>& scratch) {
  scratch.resize(L);
  expand_skew(x, L, scratch.data());
  return energy_direct(scratch.data(), L);
}

uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct WalkResult {
  int64_t best_E;
  Key best;
  int64_t steps;
  uint64_t digest;
};

// One self-avoiding walk, followed step by step (Eq. 3, Alg. 2).
WalkResult walk_one(int L, const uint64_t* start, int64_t walk_len,
                    int16_t* trace_j, int32_t* trace_E) {
  const int D = free_bits(L);
  std::vector<int8_t> x(D), y(D), scratch;
  Key start_key{};
  for (int w = 0; w < key_words(D); ++w) start_key[w] = start[w];
  unpack_key(start_key.data(), D, x.data());
  // Re-pack so stray high bits in the input never enter the visited set.
  Key cur = pack_key(x.data(), D);

  int64_t E = energy_of_free_bits(x.data(), L, scratch);
  std::set<Key> visited;
  visited.insert(cur);
  WalkResult r{E, cur, 0, 0};
  uint64_t h = 0;

  for (int64_t t = 0; t < walk_len; ++t) {
    int best_j = 0;                        // 0 = no unvisited neighbour yet
    int64_t best_e = 0;
    for (int j = 1; j <= D; ++j) {
      y = x;
      y[j - 1] = (int8_t)(-y[j - 1]);
      Key ky = pack_key(y.data(), D);
      if (visited.count(ky)) continue;
      int64_t e = energy_of_free_bits(y.data(), L, scratch);
      if (best_j == 0 || e < best_e) { best_e = e; best_j = j; }
    }
    if (best_j == 0) break;                // trapped: all D neighbours visited
    x[best_j - 1] = (int8_t)(-x[best_j - 1]);
    cur = pack_key(x.data(), D);
    E = best_e;
    visited.insert(cur);
    if (trace_j) trace_j[t] = (int16_t)best_j;
    if (trace_E) trace_E[t] = (int32_t)E;
    h = mix64(h ^ (((uint64_t)best_j << 32) | (uint64_t)(uint32_t)E));
    r.steps = t + 1;
    if (E < r.best_E) { r.best_E = E; r.best = cur; }
  }
  r.digest = mix64(h ^ (uint64_t)r.steps);
  return r;
}

// One self-avoiding walk over the whole search space: every neighbour is the
// pivot with one sequence position negated, scored by Eq. 1 directly; the
// choice, trap, best and digest rules are those of walk_one.
WalkResult walk_full_one(int L, const uint64_t* start, int64_t walk_len,
                         int16_t* trace_j, int32_t* trace_E) {
  std::vector<int8_t> s(L), y(L);
  Key start_key{};
  for (int w = 0; w < key_words(L); ++w) start_key[w] = start[w];
  unpack_key(start_key.data(), L, s.data());
  Key cur = pack_key(s.data(), L);

  int64_t E = energy_direct(s.data(), L);
  std::set<Key> visited;
  visited.insert(cur);
  WalkResult r{E, cur, 0, 0};
  uint64_t h = 0;

  for (int64_t t = 0; t < walk_len; ++t) {
    int best_i = 0;                        // 0 = no unvisited neighbour yet
    int64_t best_e = 0;
    for (int i = 1; i <= L; ++i) {
      y = s;
      y[i - 1] = (int8_t)(-y[i - 1]);
      if (visited.count(pack_key(y.data(), L))) continue;
      const int64_t e = energy_direct(y.data(), L);
      if (best_i == 0 || e < best_e) { best_e = e; best_i = i; }
    }
    if (best_i == 0) break;                // trapped: all L neighbours visited
    s[best_i - 1] = (int8_t)(-s[best_i - 1]);
    cur = pack_key(s.data(), L);
    E = best_e;
    visited.insert(cur);
    if (trace_j) trace_j[t] = (int16_t)best_i;
    if (trace_E) trace_E[t] = (int32_t)E;
    h = mix64(h ^ (((uint64_t)best_i << 32) | (uint64_t)(uint32_t)E));
    r.steps = t + 1;
    if (E < r.best_E) { r.best_E = E; r.best = cur; }
  }
  r.digest = mix64(h ^ (uint64_t)r.steps);
  return r;
}

}  // namespace

extern "C" {

int32_t orc_l_max(void) { return ORC_L_MAX; }

// Eq. 1 energy of a full +-1 sequence of any length L >= 1.
int64_t orc_energy(const int8_t* s, int32_t L) {
  if (!s || L < 1) return -1;
  return energy_direct(s, L);
}

// Eq. 2 expansion of D free bits (+-1) into the full skew-symmetric sequence.
int32_t orc_expand_skew(const int8_t* x, int32_t L, int8_t* s) {
  if (!x || !s || !valid_skew_L(L)) return -1;
  expand_skew(x, L, s);
  return 0;
}

// Energy of a packed skew-symmetric key (expand, then Eq. 1).
int64_t orc_energy_packed(const uint64_t* key, int32_t L) {
  if (!key || !valid_skew_L(L)) return -1;
  int D = free_bits(L);
  std::vector<int8_t> x(D), scratch;
  unpack_key(key, D, x.data());
  return energy_of_free_bits(x.data(), L, scratch);
}

uint64_t orc_mix64(uint64_t z) { return mix64(z); }

// Seeded uniform starts: n_walks keys of W words each, row-major.
int32_t orc_starts(int32_t L, int64_t n_walks, uint64_t seed, uint64_t* out) {
  if (!out || !valid_skew_L(L) || n_walks < 0) return -1;
  const int D = free_bits(L), W = key_words(D);
  const uint64_t G = 0x9E3779B97F4A7C15ull;
  for (int64_t w = 0; w < n_walks; ++w) {
    for (int t = 0; t < W; ++t) {
      uint64_t v = mix64(seed + G * ((uint64_t)w * (uint64_t)W + (uint64_t)t + 1u));
      int bits = D - 64 * t;
      if (bits < 64) v &= (((uint64_t)1 << bits) - 1u);
      out[w * W + t] = v;
    }
  }
  return 0;
}

// One walk.  best_seq receives W words; traces (nullable) receive one entry
// per completed move (j is 1-based, E the energy after the move).
int32_t orc_walk(int32_t L, const uint64_t* start, int64_t walk_len,
                 int64_t* best_E, uint64_t* best_seq, int64_t* steps_done,
                 uint64_t* digest, int16_t* trace_j, int32_t* trace_E) {
  if (!valid_skew_L(L) || !start || walk_len < 0) return -1;
  WalkResult r = walk_one(L, start, walk_len, trace_j, trace_E);
  const int W = key_words(free_bits(L));
  if (best_E) *best_E = r.best_E;
  if (best_seq) for (int w = 0; w < W; ++w) best_seq[w] = r.best[w];
  if (steps_done) *steps_done = r.steps;
  if (digest) *digest = r.digest;
  return 0;
}

// Many independent walks (Eq. 4) spread over n_threads host threads.
int32_t orc_walks(int32_t L, const uint64_t* starts, int64_t n_walks,
                  int64_t walk_len, int64_t* best_E, uint64_t* best_seq,
                  int64_t* steps_done, uint64_t* digest, int32_t n_threads) {
  if (!valid_skew_L(L) || !starts || n_walks < 0 || walk_len < 0) return -1;
  const int W = key_words(free_bits(L));
  if (n_threads < 1) n_threads = 1;
  std::atomic<int64_t> next{0};
  auto worker = [&]() {
    for (;;) {
      int64_t w = next.fetch_add(1);
      if (w >= n_walks) break;
      WalkResult r = walk_one(L, starts + w * W, walk_len, nullptr, nullptr);
      if (best_E) best_E[w] = r.best_E;
      if (best_seq) for (int t = 0; t < W; ++t) best_seq[w * W + t] = r.best[t];
      if (steps_done) steps_done[w] = r.steps;
      if (digest) digest[w] = r.digest;
    }
  };
  std::vector<std::thread> pool;
  for (int i = 0; i < n_threads; ++i) pool.emplace_back(worker);
  for (auto& th : pool) th.join();
  return 0;
}

// Exhaustive enumeration of all 2^D skew-symmetric sequences of length L.
// Reports the minimum energy, how many sequences attain it, the first
// minimiser (in increasing key order) and the sum of all energies.
int32_t orc_bruteforce(int32_t L, int64_t* min_E, int64_t* n_min,
                       uint64_t* first_min_key, int64_t* sum_E) {
  if (!valid_skew_L(L)) return -1;
  const int D = free_bits(L);
  if (D > 30) return -1;
  std::vector<int8_t> x(D), scratch;
  int64_t best = -1, count = 0, total = 0;
  uint64_t first = 0;
  for (uint64_t v = 0; v < ((uint64_t)1 << D); ++v) {
    unpack_key(&v, D, x.data());
    int64_t e = energy_of_free_bits(x.data(), L, scratch);
    total += e;
    if (best < 0 || e < best) { best = e; count = 1; first = v; }
    else if (e == best) ++count;
  }
  if (min_E) *min_E = best;
  if (n_min) *n_min = count;
  if (first_min_key) *first_min_key = first;
  if (sum_E) *sum_E = total;
  return 0;
}

// ---- the whole search space -------------------------------------------

int32_t orc_full_l_max(void) { return ORC_FULL_L_MAX; }

// Seeded uniform starts over all L positions: W = ceil(L/64) words per walk.
int32_t orc_full_starts(int32_t L, int64_t n_walks, uint64_t seed, uint64_t* out) {
  if (!out || !valid_full_L(L) || n_walks < 0) return -1;
  const int W = key_words(L);
  const uint64_t G = 0x9E3779B97F4A7C15ull;
  for (int64_t w = 0; w < n_walks; ++w) {
    for (int t = 0; t < W; ++t) {
      uint64_t v = mix64(seed + G * ((uint64_t)w * (uint64_t)W + (uint64_t)t + 1u));
      int bits = L - 64 * t;
      if (bits < 64) v &= (((uint64_t)1 << bits) - 1u);
      out[w * W + t] = v;
    }
  }
  return 0;
}

// Eq. 1 energy of a packed whole sequence (bit i-1 = s_i, 1 means -1).
int64_t orc_full_energy_packed(const uint64_t* key, int32_t L) {
  if (!key || !valid_full_L(L)) return -1;
  std::vector<int8_t> s(L);
  unpack_key(key, L, s.data());
  return energy_direct(s.data(), L);
}

int32_t orc_full_walk(int32_t L, const uint64_t* start, int64_t walk_len,
                      int64_t* best_E, uint64_t* best_seq, int64_t* steps_done,
                      uint64_t* digest, int16_t* trace_j, int32_t* trace_E) {
  if (!valid_full_L(L) || !start || walk_len < 0) return -1;
  WalkResult r = walk_full_one(L, start, walk_len, trace_j, trace_E);
  const int W = key_words(L);
  if (best_E) *best_E = r.best_E;
  if (best_seq) for (int w = 0; w < W; ++w) best_seq[w] = r.best[w];
  if (steps_done) *steps_done = r.steps;
  if (digest) *digest = r.digest;
  return 0;
}

int32_t orc_full_walks(int32_t L, const uint64_t* starts, int64_t n_walks,
                       int64_t walk_len, int64_t* best_E, uint64_t* best_seq,
                       int64_t* steps_done, uint64_t* digest, int32_t n_threads) {
  if (!valid_full_L(L) || !starts || n_walks < 0 || walk_len < 0) return -1;
  const int W = key_words(L);
  if (n_threads < 1) n_threads = 1;
  std::atomic<int64_t> next{0};
  auto worker = [&]() {
    for (;;) {
      int64_t w = next.fetch_add(1);
      if (w >= n_walks) break;
      WalkResult r = walk_full_one(L, starts + w * W, walk_len, nullptr, nullptr);
      if (best_E) best_E[w] = r.best_E;
      if (best_seq) for (int t = 0; t < W; ++t) best_seq[w * W + t] = r.best[t];
      if (steps_done) steps_done[w] = r.steps;
      if (digest) digest[w] = r.digest;
    }
  };
  std::vector<std::thread> pool;
  for (int i = 0; i < n_threads; ++i) pool.emplace_back(worker);
  for (auto& th : pool) th.join();
  return 0;
}

// Exhaustive enumeration of all 2^L sequences of length L (L <= 26): minimum
// energy, number of minimisers, first minimiser (increasing key order) and
// the sum of all energies.
int32_t orc_full_bruteforce(int32_t L, int64_t* min_E, int64_t* n_min,
                            uint64_t* first_min_key, int64_t* sum_E) {
  if (L < 1 || L > 26) return -1;
  std::vector<int8_t> s(L);
  int64_t best = -1, count = 0, total = 0;
  uint64_t first = 0;
  for (uint64_t v = 0; v < ((uint64_t)1 << L); ++v) {
    unpack_key(&v, L, s.data());
    const int64_t e = energy_direct(s.data(), L);
    total += e;
    if (best < 0 || e < best) { best = e; count = 1; first = v; }
    else if (e == best) ++count;
  }
  if (min_E) *min_E = best;
  if (n_min) *n_min = count;
  if (first_min_key) *first_min_key = first;
  if (sum_E) *sum_E = total;
  return 0;
}

}  // extern "C"
