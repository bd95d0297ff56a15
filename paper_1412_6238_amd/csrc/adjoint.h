// adjoint.h -- checkpoint storage for reverse-mode differentiation of a
// recorded run (layout and checkpoint copies).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

namespace lbe {

struct AdjLayout {
  int64_t record_steps;   // capacity N
  int64_t K;              // checkpoint spacing ceil(sqrt(N))
  int64_t nchk;           // checkpoints ceil(N / K)
  size_t state_bytes;
  size_t off_chk;         // nchk states
  size_t off_tape;        // K states (one segment replayed)
  size_t off_lam;         // two adjoint states (FP64 or FP32 like the state)
  size_t off_part;        // per-block FP64 partials of dJ/dsigmaT
  size_t off_tw;          // FP64 [2][nx] accumulators for dJ/dTwall
  size_t total;
};

inline int64_t adj_segment_length(int64_t nsteps) {
  if (nsteps <= 0) return 1;
  int64_t K = (int64_t)std::ceil(std::sqrt((double)nsteps));
  while (K * K < nsteps) ++K;
  return K < 1 ? 1 : K;
}

inline AdjLayout adj_layout(int nx, size_t state_bytes, int nblocks, int64_t record_steps) {
  AdjLayout A{};
  auto al = [](size_t v) { return (v + 255) / 256 * 256; };
  A.record_steps = record_steps;
  if (record_steps <= 0) return A;
  A.state_bytes = al(state_bytes);
  A.K = adj_segment_length(record_steps);
  A.nchk = (record_steps + A.K - 1) / A.K;
  size_t o = 0;
  A.off_chk = o; o += (size_t)A.nchk * A.state_bytes;
  A.off_tape = o; o += (size_t)A.K * A.state_bytes;
  A.off_lam = o; o += 2 * A.state_bytes;
  A.off_part = o; o += al((size_t)nblocks * 8 * sizeof(double));
  A.off_tw = o; o += al(2 * (size_t)nx * sizeof(double));
  A.total = o;
  return A;
}

inline int adj_save_checkpoint(char *adj_base, const AdjLayout &A, int64_t k,
                               const void *state, size_t bytes, hipStream_t st) {
  if (k < 0 || k >= A.nchk) return 1;
  char *dst = adj_base + A.off_chk + (size_t)k * A.state_bytes;
  return hipMemcpyAsync(dst, state, bytes, hipMemcpyDeviceToDevice, st) == hipSuccess ? 0 : 1;
}

}  // namespace lbe
