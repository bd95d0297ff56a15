// lattice.h -- D2Q9 tables and the per-launch argument block shared by the
// forward and adjoint kernels of liblbe_csf.
//
// The velocity set, weights and opposite directions are those implied by the
// weights of the equilibria in Sec. II (Eqs. 7-8, 13-14) of arXiv:1412.6238:
// rest weight 4/9, axis 1/9, diagonal 1/36, cs^2 = 1/3.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "host_layout.h"

namespace lbe {

constexpr int kQ = 9;
constexpr int kEx[kQ] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int kEy[kQ] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int kOpp[kQ] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

template <typename R>
__host__ __device__ constexpr R wq(int i) {
  return i == 0 ? R(4) / R(9) : (i < 5 ? R(1) / R(9) : R(1) / R(36));
}

// Kernel modes (bit set).
enum : int {
  kStore = 1,   // collide and stream into dst
  kFields = 2,  // write phi, u, p, T
  kDiag = 4,    // per-block FP64 partial sums of the diagnostics
  kTape = 8,    // write the moments of the source state to the tape
  kCurv = 16,   // capillary force in the curvature form of Eq. 4
  kVarRho = 32, // two densities, rho(c) = rho + c drho
  kPress = 64,  // with kVarRho: only the pressure of Eq. 9, into a plane
  kStream = 128 // FP32 form, state larger than the last-level cache: stores
                // that write whole lines bypass that cache (buf_store_stream)
};

// Everything a step launch needs, passed by value.  Derived constants are
// computed once on the host in FP64 and rounded to the kernel's arithmetic
// type inside the kernel.
struct StepArgs {
  const void *src;
  void *dst;
  int nx, ny, walls_y;
  int nstrips, rows_per_chunk;
  const double *twb, *twt;  // wall temperatures [nx]
  // physical and derived constants
  double rho, cv, rcv;      // rho, cv, rho*cv
  double tauf0, dtauf;      // tau_f(c) = tauf0 + clamp(c) dtauf
  double tauT0, dtauT;
  double omg_g;             // 1 / tau_g
  double gam3;              // Gamma / cs^2 = 3 Gamma
  double beta2;             // 2 beta  (mu0 = 2 beta c (c-1)(2c-1))
  double eps2;              // eps^2
  double kcap, epsalpha;    // alpha/eps and eps*alpha
  double sigma0, sigmaT, Tref;
  double ax, ay;            // body acceleration
  double p0, Ts, Tg;        // deviation references (FP32 form): w p0 for f,
                            // w rho cv (Ts + Tg y) for hbar at height y
  double drho;              // rho(c) = rho + c drho (kVarRho)
  const double *pc;         // kVarRho: the pressure of Eq. 9 of the source
                            // state, p = sum f + (1/2) u.grad(rho cs^2)
  double *pc_out;           // kPress: where that pressure is written
  // outputs
  double *phi, *ux, *uy, *p, *T;
  double *partials;         // [gridDim.x][kNumPartials]
  // moment tape of the source state (kTape; read by the adjoint): c as FP64,
  // then T, p, jx, jy in the arithmetic type (T and p as deviations in the
  // FP32 form), each a plane of nx*ny
  void *tape;
};

// Buffer resources: one descriptor per buffer (scalar registers) and a 32-bit
// byte offset per lane, so a load or store needs one vector register for its
// address instead of two.  The third descriptor word 0x00020000 is the CDNA
// (gfx9 family) raw-buffer format; accesses past num_records return zero /
// are dropped instead of faulting.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void *base, size_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                           0x00020000);
}

// byte_off: per-lane offset (vector register); base: uniform offset (scalar
// register), e.g. a plane's segment within a row of the state
template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t byte_off,
                                      uint32_t base = 0) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)byte_off,
                                                                       (int)base, 0));
  } else {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)byte_off,
                                                                       (int)base, 0));
  }
}

// Stores use the default cache policy: measured on MI355X, marking these
// (shifted, partially overlapping) row stores non-temporal made the step
// slower, because neighbouring waves' partial lines then reach HBM unmerged.
template <typename T>
__device__ __forceinline__ void buf_store(T v, __amdgpu_buffer_rsrc_t r, uint32_t byte_off,
                                             uint32_t base = 0) {
  if constexpr (sizeof(T) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)byte_off,
                                          (int)base, 0);
  } else {
    using V2 = __attribute__((ext_vector_type(2))) uint32_t;
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), r, (int)byte_off,
                                          (int)base, 0);
  }
}

// The same store marked non-temporal.  With kStream the FP32 step uses it for
// the stores whose lines one wave writes whole (the rest populations and the
// moves along y): the lines then go to HBM without displacing the lines that
// the shifted stores of neighbouring waves are still merging.  Measured on
// 4096^2: 1.3-1.7% faster; on a 512 x 1024 grid, whose two states fit in the
// MI355X's 256 MB last-level cache, 5-9% slower, hence the size test on the
// host.
template <typename T>
__device__ __forceinline__ void buf_store_stream(T v, __amdgpu_buffer_rsrc_t r, uint32_t byte_off,
                                                 uint32_t base = 0) {
  if constexpr (sizeof(T) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)byte_off,
                                          (int)base, 2);
  } else {
    using V2 = __attribute__((ext_vector_type(2))) uint32_t;
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), r, (int)byte_off,
                                          (int)base, 2);
  }
}

// Map the hardware block index to a logical tile so that consecutive tiles
// run on the same XCD: blocks are dealt to the 8 XCDs round-robin, so XCD k
// receives a contiguous range of logical tiles (neighbouring strips and
// chunks, which share halo rows and columns, then share an L2).
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int xcd = b & 7, idx = b >> 3;
  return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

}  // namespace lbe
