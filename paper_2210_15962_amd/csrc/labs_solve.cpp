// labs_solve.cpp -- the solver driver (Alg. 1) and the stopping model of
// Sec. 4 (Eq. 6, Eq. 7) of liblabs.so.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <chrono>
#include <limits>
#include <vector>

#include "labs.h"
#include "labs_internal.h"

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;   // SplitMix64 increment
constexpr double kLambdaA = 0.006753;                // lambda(L) = A * B^L, Sec. 4
constexpr double kLambdaB = 0.8617;

uint64_t al(uint64_t x) { return (x + 255) & ~(uint64_t)255; }

bool valid_L(int32_t L) { return L >= 3 && L <= lsaw::kLMax && (L & 1); }

struct SolveLayout {
  int64_t n = 0, walk_len = 0;
  int W = 0;
  uint64_t tables = 0, off_E = 0, off_steps = 0, off_seq = 0, total = 0;
};

int32_t layout(int32_t L, const labs_solve_cfg *c, SolveLayout &o) {
  if (!valid_L(L)) return lsaw::set_error(LABS_EINVAL, "L=%d: need odd L with 3 <= L <= %d", L, lsaw::kLMax);
  if (!c) return lsaw::set_error(LABS_EINVAL, "NULL configuration");
  if (c->walks_per_round <= 0) return lsaw::set_error(LABS_EINVAL, "walks_per_round must be > 0");
  if (c->walk_len < 0) return lsaw::set_error(LABS_EINVAL, "walk_len must be >= 0");
  if (c->time_limit_s < 0 || c->nses_limit < 0 || c->max_rounds < 0 || c->target_E < 0)
    return lsaw::set_error(LABS_EINVAL, "negative stopping limit");
  if (c->first_round < 0) return lsaw::set_error(LABS_EINVAL, "first_round must be >= 0");
  if (!(c->time_limit_s > 0 || c->nses_limit > 0 || c->max_rounds > 0 || c->target_E > 0))
    return lsaw::set_error(LABS_EINVAL, "no stopping condition (time, NSEs, target or rounds)");
  const int D = lsaw::free_bits(L);
  o.n = c->walks_per_round;
  o.walk_len = c->walk_len ? c->walk_len : 8 * (int64_t)D;
  o.W = lsaw::key_words_for(L);
  uint64_t tb = 0;
  int32_t rc = labs_walks_workspace_bytes(L, o.n, o.walk_len, &c->plan, &tb);
  if (rc != LABS_OK) return rc;
  o.tables = al(tb);
  o.off_E = o.tables;
  o.off_steps = o.off_E + al((uint64_t)o.n * 4);
  o.off_seq = o.off_steps + al((uint64_t)o.n * 8);
  o.total = o.off_seq + al((uint64_t)o.n * 8 * o.W);
  return LABS_OK;
}

double elapsed_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

extern "C" {

int32_t labs_solve_workspace_bytes(int32_t L, const labs_solve_cfg *cfg, uint64_t *bytes) {
  if (!bytes) return lsaw::set_error(LABS_EINVAL, "NULL bytes");
  SolveLayout o;
  const int32_t rc = layout(L, cfg, o);
  if (rc != LABS_OK) return rc;
  *bytes = o.total;
  return lsaw::clear_error();
}

int32_t labs_solve(int32_t L, const labs_solve_cfg *cfg, void *workspace, uint64_t ws_bytes,
                   void *stream, labs_solve_result *res) {
  if (!res) return lsaw::set_error(LABS_EINVAL, "NULL result");
  SolveLayout o;
  int32_t rc = layout(L, cfg, o);
  if (rc != LABS_OK) return rc;
  if (!workspace) return lsaw::set_error(LABS_EINVAL, "NULL workspace");
  if (ws_bytes < o.total)
    return lsaw::set_error(LABS_EINVAL, "workspace of %llu bytes is below the %llu needed",
                           (unsigned long long)ws_bytes, (unsigned long long)o.total);
  const int D = lsaw::free_bits(L);
  uint8_t *ws = static_cast<uint8_t *>(workspace);
  int32_t *dE = reinterpret_cast<int32_t *>(ws + o.off_E);
  int64_t *dsteps = reinterpret_cast<int64_t *>(ws + o.off_steps);
  uint64_t *dseq = reinterpret_cast<uint64_t *>(ws + o.off_seq);
  hipStream_t st = static_cast<hipStream_t>(stream);
  labs_walk_out out{dseq, dE, dsteps, nullptr, nullptr, nullptr, 0, nullptr};
  std::vector<int32_t> hE((size_t)o.n);
  std::vector<int64_t> hsteps((size_t)o.n);

  *res = labs_solve_result{};
  res->best_E = std::numeric_limits<int32_t>::max();
  res->target_seconds = -1.0;
  res->target_nfes = -1.0;
  const auto t0 = std::chrono::steady_clock::now();
  const double nfes_per_round = (double)o.n * (double)o.walk_len * (double)(D - 1);
  for (int64_t r = 0;; ++r) {
    if (cfg->max_rounds > 0 && r >= cfg->max_rounds) break;
    if (cfg->time_limit_s > 0 && elapsed_s(t0) >= cfg->time_limit_s) break;
    if (cfg->nses_limit > 0 && res->nfes >= cfg->nses_limit) break;
    if (res->reached_target) break;
    // walks q*n .. q*n + n - 1 of the seed's start stream, q = first_round + r
    const uint64_t q = (uint64_t)cfg->first_round + (uint64_t)r;
    const uint64_t seed_r = cfg->seed + kGamma * (q * (uint64_t)o.n * (uint64_t)o.W);
    rc = labs_walks(nullptr, L, o.n, o.walk_len, seed_r, &out, ws, o.tables, &cfg->plan, stream);
    if (rc != LABS_OK) return rc;
    hipError_t e = hipMemcpyAsync(hE.data(), dE, hE.size() * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(hsteps.data(), dsteps, hsteps.size() * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return lsaw::set_error(LABS_EDEVICE, "solve round: %s", hipGetErrorString(e));
    res->rounds = r + 1;
    res->nfes += nfes_per_round;
    for (int64_t v : hsteps) res->walk_steps += (double)v;
    int64_t b = 0;
    for (int64_t i = 1; i < o.n; ++i)
      if (hE[(size_t)i] < hE[(size_t)b]) b = i;       // first walk of the round's minimum
    if (hE[(size_t)b] < res->best_E) {
      res->best_E = hE[(size_t)b];
      uint64_t seq[3] = {0, 0, 0};
      e = hipMemcpyAsync(seq, dseq + (uint64_t)b * o.W, (size_t)o.W * 8, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) return lsaw::set_error(LABS_EDEVICE, "solve copy: %s", hipGetErrorString(e));
      for (int t = 0; t < 3; ++t) res->best_seq[t] = seq[t];
    }
    if (cfg->target_E > 0 && res->best_E <= cfg->target_E && !res->reached_target) {
      res->reached_target = 1;
      res->target_seconds = elapsed_s(t0);
      res->target_nfes = res->nfes;
    }
  }
  res->seconds = elapsed_s(t0);
  return lsaw::clear_error();
}

double labs_lambda_model(int32_t L) {
  if (L < 1) return NAN;
  return kLambdaA * pow(kLambdaB, (double)L);
}

double labs_nses_limit(int32_t L, double P, int32_t N) {
  if (L < 1 || !(P > 0.0 && P < 1.0) || N < 1) return NAN;
  return log(1.0 - P) / (-labs_lambda_model(L) * (double)N);
}

double labs_optimality_probability(int32_t L, double nses_total) {
  if (L < 1 || !(nses_total >= 0.0)) return NAN;
  return 1.0 - exp(-labs_lambda_model(L) * nses_total);
}

}  // extern "C"
