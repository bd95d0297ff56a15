// aux_kernels.h -- initial state, diagnostic reduction and state conversion.
#pragma once

#include "lattice.h"
#include "step_kernel.h"

namespace lbe {

// Initial state: u = 0, p = p0, c0 = (1 + phi0)/2, mu0 from c0 and its
// nine-point Laplacian (mirror ghosts at walls), every distribution at its
// equilibrium (Sec. II Eqs. 7, 13-14; Sec. III Eq. 22).  FP32 form: stored as
// deviations, so f - w p0 = 0 and hbar - w rho cv Tr = w rho cv (T0 - Tr)
// with the linear reference Tr = Ts + Tg (y + 1/2) of the site's row.
// Layout as in host_layout.h: rows of 25 plane segments of S, then the rest
// populations g_0 and hbar_0.
template <typename S, bool DEV>
__global__ void __launch_bounds__(256)
init_kernel(S *__restrict__ F, const double *__restrict__ phi0,
            const double *__restrict__ T0, int nx, int ny, int walls_y,
            double beta2, double eps2, double gam3, double rcv, double p0,
            double Ts, double Tg, double rho, double drho, double cv) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= nx || y >= ny) return;
  const size_t s = (size_t)y * nx + x;
  auto cval = [&](int dx, int dy) {
    int xx = x + dx;
    xx = xx < 0 ? xx + nx : (xx >= nx ? xx - nx : xx);
    int yy = y + dy;
    if (walls_y) {
      yy = yy < 0 ? 0 : (yy >= ny ? ny - 1 : yy);  // mirror of a ghost row
    } else {
      yy = yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy);
    }
    return 0.5 * (1.0 + phi0[(size_t)yy * nx + xx]);
  };
  const double c = cval(0, 0);
  const double lap = (2.0 / 3.0) * ((cval(1, 0) - c) + (cval(-1, 0) - c) + (cval(0, 1) - c) +
                                    (cval(0, -1) - c)) +
                     (1.0 / 6.0) * ((cval(1, 1) - c) + (cval(-1, 1) - c) + (cval(1, -1) - c) +
                                    (cval(-1, -1) - c));
  const double mu = beta2 * c * (c - 1.0) * (2.0 * c - 1.0) - eps2 * lap;
  const double gmu = gam3 * mu;
  const double T = T0[s];
  const double Tr = Ts + Tg * (y + 0.5);
  // two densities: rho(c) cv of the site (rcv itself with one density); the
  // FP32 form's reference keeps the density of the c = 0 fluid
  const double rcv_s = drho != 0.0 ? (rho + c * drho) * cv : rcv;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const double w = wq<double>(i);
    F[plane_index<S>(plane_of(i), nx, y, x)] = DEV ? S(0) : S(w * p0);
    const double hv = DEV ? (drho != 0.0 ? w * (rcv_s * T - rcv * Tr) : w * rcv * (T - Tr))
                          : w * rcv_s * T;
    if (i == 0) {
      rest_set<S, 0>(F, nx, y, x, c - (1.0 - w) * gmu);
      rest_set<S, 1>(F, nx, y, x, hv);
    } else {
      F[plane_index<S>(plane_of(9 + i), nx, y, x)] = S(w * gmu);
      F[plane_index<S>(plane_of(18 + i), nx, y, x)] = S(hv);
    }
  }
}

// Deterministic final reduction of the per-block partials into one record,
// appended to a device ring of records (DiagRecord, host_layout.h).

__global__ void __launch_bounds__(256)
diag_reduce_kernel(const double *__restrict__ partials, int nblocks,
                   DiagRecord *__restrict__ ring, int ring_cap,
                   int64_t *__restrict__ counters, int64_t step) {
  __shared__ double s[kNumPartials][256];
  const int t = threadIdx.x;
  double acc[kNumPartials];
#pragma unroll
  for (int k = 0; k < kNumPartials; ++k) acc[k] = 0.0;
  for (int b = t; b < nblocks; b += 256) {
#pragma unroll
    for (int k = 0; k < kNumPartials; ++k) acc[k] += partials[(size_t)b * kNumPartials + k];
  }
#pragma unroll
  for (int k = 0; k < kNumPartials; ++k) s[k][t] = acc[k];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
#pragma unroll
      for (int k = 0; k < kNumPartials; ++k) s[k][t] += s[k][t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    // With counters: append to the ring (counters[0]: records written so
    // far, counters[1]: non-finite total).  Without: write ring[0].
    const int64_t idx = counters ? counters[0] : 0;
    DiagRecord &r = ring[idx % ring_cap];
    r.step = step;
#pragma unroll
    for (int k = 0; k < kNumPartials; ++k) r.v[k] = s[k][0];
    if (counters) {
      counters[0] = idx + 1;
      counters[1] += (int64_t)s[kNumPartials - 1][0];
    }
  }
}

// FP64 [27][n] <-> storage form (row-interleaved, host_layout.h).
template <typename S, bool DEV>
__global__ void __launch_bounds__(256)
state_to_f64(const S *__restrict__ F, double *__restrict__ out, int nx, int ny,
             double p0, double rcv, double Ts, double Tg) {
  const size_t n = (size_t)nx * ny;
  const size_t s = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (s >= n) return;
  const int i = q % 9;
  const size_t y = s / nx, x = s % nx;
  double v = q == 9 ? rest_get<S, 0>(F, nx, y, x)
                    : (q == 18 ? rest_get<S, 1>(F, nx, y, x)
                               : double(F[plane_index<S>(plane_of(q), nx, y, x)]));
  if (DEV) {
    if (q < 9) v += wq<double>(i) * p0;
    else if (q >= 18) v += wq<double>(i) * rcv * (Ts + Tg * (double(y) + 0.5));
  }
  out[q * n + s] = v;
}

template <typename S, bool DEV>
__global__ void __launch_bounds__(256)
state_from_f64(S *__restrict__ F, const double *__restrict__ in, int nx, int ny,
               double p0, double rcv, double Ts, double Tg) {
  const size_t n = (size_t)nx * ny;
  const size_t s = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (s >= n) return;
  const int i = q % 9;
  const size_t y = s / nx, x = s % nx;
  double v = in[q * n + s];
  if (DEV) {
    if (q < 9) v -= wq<double>(i) * p0;
    else if (q >= 18) v -= wq<double>(i) * rcv * (Ts + Tg * (double(y) + 0.5));
  }
  if (q == 9) rest_set<S, 0>(F, nx, y, x, v);
  else if (q == 18) rest_set<S, 1>(F, nx, y, x, v);
  else F[plane_index<S>(plane_of(q), nx, y, x)] = S(v);
}

}  // namespace lbe
