// CFL time step of Sec. 2.5, reduced on the device in two passes.
//
// Per cell: conv = min(dx/(|u|+c), dy/(|v|+c)) and visc = min(dx^2/nu, dy^2/nu)
// (nu = mu/rho), each evaluated with one rounding per operation and IEEE
// division / square root.  Pass 1: every workgroup reduces its cells to one
// (conv, visc) pair in a fixed grid-stride pattern; pass 2: one workgroup
// reduces the pairs and writes dt = cfl * min(visc / alpha_v, conv).  A min
// is exact, so the result is bit-identical to any other evaluation order; no
// atomics are used.  A bad cell (non-finite, rho <= 0, p <= 0) is recorded
// in the status word, since fmin would otherwise drop a NaN.
#pragma once
#include "stage_kernel.hpp"

namespace gbr {

constexpr int kDtBlocks = 1024;  // pass-1 workgroups at most (partials kept in context scratch)
constexpr int kDtThreads = 256;

// Pass-1 workgroups for n cells: 1024 from 4M cells on, where more loads in
// flight pay (-17% at 4096^2); 512 below, where the second pass's extra
// partials would cost more than they save.
inline int dt_blocks(size_t n) {
  const size_t want = (n + kDtThreads - 1) / kDtThreads;
  const size_t cap = n >= (size_t(1) << 22) ? kDtBlocks : kDtBlocks / 2;
  return (int)(want < cap ? want : cap);
}

struct DtParams {
  const double* __restrict__ Q;
  double* partial;   // [2][kDtBlocks] (context scratch holds [3][kDtBlocks])
  double* dt;
  unsigned* status;
  int nx, ny;
  double dx, dy, gamma, mu, cfl;
};

__device__ __forceinline__ double block_min(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if (__lane_id() == 0) red[w] = v;
  __syncthreads();
  double r = red[0];
  for (int k = 1; k < (int)(blockDim.x >> 6); ++k) r = fmin(r, red[k]);
  return r;
}

// Convective and viscous limits of cell s folded into (conv, visc).
__device__ __forceinline__ void dt_cell(const double* __restrict__ Q, size_t n, size_t s,
                                        double gamma, double mu, double dx, double dy,
                                        double& conv, double& visc, bool& bad) {
#pragma clang fp contract(off)
  const double rho = Q[s];
  const double u = Q[n + s] / rho, v = Q[2 * n + s] / rho;
  const double p = (gamma - 1.0) * (Q[3 * n + s] - rho * (u * u + v * v) / 2.0);
  const double c = sqrt(gamma * p / rho);
  if (!(rho > 0.0) || !(p > 0.0) || !isfinite(c) || !isfinite(u) || !isfinite(v)) bad = true;
  conv = fmin(conv, fmin(dx / (fabs(u) + c), dy / (fabs(v) + c)));
  if (mu > 0.0) {
    const double nu = mu / rho;
    visc = fmin(visc, fmin(dx * dx / nu, dy * dy / nu));
  }
}

__global__ __launch_bounds__(kDtThreads) void dt_reduce_kernel(DtParams P) {
#pragma clang fp contract(off)
  __shared__ double red[kDtThreads / 64];
  const size_t n = (size_t)P.nx * P.ny;
  double conv = __builtin_inf(), visc = __builtin_inf();
  bool bad = false;
  for (size_t s = (size_t)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (size_t)gridDim.x * blockDim.x) {
    dt_cell(P.Q, n, s, P.gamma, P.mu, P.dx, P.dy, conv, visc, bad);
  }
  if (bad) atomicOr(P.status, 1u);
  conv = block_min(conv, red);
  visc = block_min(visc, red);
  if (threadIdx.x == 0) {
    P.partial[blockIdx.x] = conv;
    P.partial[kDtBlocks + blockIdx.x] = visc;
  }
}

__global__ __launch_bounds__(kDtThreads) void dt_finish_kernel(const double* partial, int nblk,
                                                               double* dt, double cfl,
                                                               unsigned* status) {
#pragma clang fp contract(off)
  __shared__ double red[kDtThreads / 64];
  double conv = __builtin_inf(), visc = __builtin_inf();
  for (int k = threadIdx.x; k < nblk; k += blockDim.x) {
    conv = fmin(conv, partial[k]);
    visc = fmin(visc, partial[kDtBlocks + k]);
  }
  conv = block_min(conv, red);
  visc = block_min(visc, red);
  if (threadIdx.x == 0) {
    const double d = cfl * fmin(visc / kAlphaV, conv);
    *dt = d;
    if (!(d > 0.0) || !isfinite(d)) atomicOr(status, 2u);
  }
}

// Second pass of the time step without a context: as dt_finish_kernel, with
// the status word in the same scratch as the partials.  A bad state seen by
// the first pass makes dt NaN (the caller has no context to ask), and the
// word is cleared for the next call.
__global__ __launch_bounds__(kDtThreads) void dt_finish_noalloc_kernel(const double* partial,
                                                                       int nblk, double* dt,
                                                                       double cfl,
                                                                       unsigned* status) {
#pragma clang fp contract(off)
  __shared__ double red[kDtThreads / 64];
  double conv = __builtin_inf(), visc = __builtin_inf();
  for (int k = threadIdx.x; k < nblk; k += blockDim.x) {
    conv = fmin(conv, partial[k]);
    visc = fmin(visc, partial[kDtBlocks + k]);
  }
  conv = block_min(conv, red);
  visc = block_min(visc, red);
  if (threadIdx.x == 0) {
    const double d = cfl * fmin(visc / kAlphaV, conv);
    *dt = (*status != 0u) ? __builtin_nan("") : d;
    *status = 0u;
  }
}

// dt from the extrema the stage-3 kernel left per workgroup, in two passes
// like the reduction above: pass 1 folds the slots [3][nslot] into
// kDtBlocks partial extrema, pass 2 (one workgroup) finishes with the
// arithmetic of dt_cell and dt_finish_kernel -- the minimum over cells of
// fl(dx/(|u|+c)) is fl(dx/max(|u|+c)), and that of fl(fl(dx dx)/fl(mu/rho))
// is fl(fl(dx dx)/fl(mu/min rho)), since fl(d/x) is monotone in x.
__device__ __forceinline__ double block_max(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if (__lane_id() == 0) red[w] = v;
  __syncthreads();
  double r = red[0];
  for (int k = 1; k < (int)(blockDim.x >> 6); ++k) r = fmax(r, red[k]);
  return r;
}

// MAX3: the third extremum is a maximum (3D: max(|w|+c)), else a minimum
// (2D: min rho).
template <bool MAX3 = false>
__global__ __launch_bounds__(kDtThreads) void dt_extrema_reduce_kernel(const double* slots,
                                                                       int nslot,
                                                                       double* partial) {
  __shared__ double red[kDtThreads / 64];
  double a = 0.0, b = 0.0, r = MAX3 ? 0.0 : __builtin_inf();
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nslot; k += gridDim.x * blockDim.x) {
    a = fmax(a, slots[k]);
    b = fmax(b, slots[nslot + k]);
    r = MAX3 ? fmax(r, slots[2 * nslot + k]) : fmin(r, slots[2 * nslot + k]);
  }
  a = block_max(a, red);
  b = block_max(b, red);
  r = MAX3 ? block_max(r, red) : block_min(r, red);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = a;
    partial[kDtBlocks + blockIdx.x] = b;
    partial[2 * kDtBlocks + blockIdx.x] = r;
  }
}

__global__ __launch_bounds__(kDtThreads) void dt_from_extrema_kernel(const double* partial,
                                                                     int nblk, double* dt,
                                                                     double cfl, double dx,
                                                                     double dy, double mu,
                                                                     unsigned* status) {
#pragma clang fp contract(off)
  __shared__ double red[kDtThreads / 64];
  double a = 0.0, b = 0.0, r = __builtin_inf();
  for (int k = threadIdx.x; k < nblk; k += blockDim.x) {
    a = fmax(a, partial[k]);
    b = fmax(b, partial[kDtBlocks + k]);
    r = fmin(r, partial[2 * kDtBlocks + k]);
  }
  a = block_max(a, red);
  b = block_max(b, red);
  r = block_min(r, red);
  if (threadIdx.x == 0) {
    const double conv = fmin(dx / a, dy / b);
    double visc = __builtin_inf();
    if (mu > 0.0) {
      const double nu = mu / r;
      visc = fmin(dx * dx / nu, dy * dy / nu);
    }
    const double d = cfl * fmin(visc / kAlphaV, conv);
    *dt = d;
    if (!(d > 0.0) || !isfinite(d)) atomicOr(status, 2u);
  }
}

// 3D (inviscid): dt = cfl min(dx/a, dy/b, dz/c) from the partial maxima of
// |u|+c, |v|+c, |w|+c, with the arithmetic of dt3_reduce_kernel and
// dt_finish_kernel.
__global__ __launch_bounds__(kDtThreads) void dt3_from_extrema_kernel(const double* partial,
                                                                      int nblk, double* dt,
                                                                      double cfl, double dx,
                                                                      double dy, double dz,
                                                                      unsigned* status) {
#pragma clang fp contract(off)
  __shared__ double red[kDtThreads / 64];
  double a = 0.0, b = 0.0, c = 0.0;
  for (int k = threadIdx.x; k < nblk; k += blockDim.x) {
    a = fmax(a, partial[k]);
    b = fmax(b, partial[kDtBlocks + k]);
    c = fmax(c, partial[2 * kDtBlocks + k]);
  }
  a = block_max(a, red);
  b = block_max(b, red);
  c = block_max(c, red);
  if (threadIdx.x == 0) {
    const double conv = fmin(dx / a, fmin(dy / b, dz / c));
    const double d = cfl * fmin(__builtin_inf() / kAlphaV, conv);
    *dt = d;
    if (!(d > 0.0) || !isfinite(d)) atomicOr(status, 2u);
  }
}

// Self-test of div_rb (the shared-reciprocal quotient of the time-step
// extrema) against IEEE division: `count` operand pairs drawn from a
// counter-based hash (splitmix64 of seed + index), magnitudes log-uniform over
// [2^-300, 2^300] with random signs, every 16th numerator zero; a zero
// quotient may differ in sign only.
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}
__device__ __forceinline__ double selftest_operand(unsigned long long h) {
  // exponent in [-300, 299], 52 random mantissa bits, random sign
  const long long e = (long long)((h >> 53) % 600ull) - 300;
  const unsigned long long bits = ((unsigned long long)(e + 1023) << 52) |
                                  (h & 0x000FFFFFFFFFFFFFull) | ((h >> 52 & 1ull) << 63);
  return __longlong_as_double((long long)bits);
}
__global__ __launch_bounds__(256) void div_selftest_kernel(unsigned long long seed,
                                                           unsigned long long count,
                                                           unsigned long long* bad_count) {
  const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
  unsigned long long bad = 0;
  for (unsigned long long k = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
       k < count; k += stride) {
    const unsigned long long h1 = splitmix64(seed + 2 * k), h2 = splitmix64(seed + 2 * k + 1);
    const double a = (k % 16 == 15) ? 0.0 : selftest_operand(h1);
    const double b = selftest_operand(h2);
    const double q = div_rb(a, b, rcp_nr(b)), ref = a / b;
    const bool same = __double_as_longlong(q) == __double_as_longlong(ref) ||
                      (q == 0.0 && ref == 0.0);
    if (!(div_rb_ok(a) && div_rb_ok(b)) || !same) ++bad;
  }
  if (bad) atomicAdd(bad_count, bad);
}

// t += dt on the device (the clock of moving boundary segments).
__global__ void advance_time_kernel(double* t, const double* dt) {
  if (threadIdx.x == 0) *t = *t + *dt;
}

}  // namespace gbr
