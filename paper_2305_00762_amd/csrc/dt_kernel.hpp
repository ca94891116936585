// CFL time step of Sec. 2.5, reduced on the device.
//
// Per cell: conv = min(dx/(|u|+c), dy/(|v|+c)) and visc = min(dx^2/nu, dy^2/nu)
// (nu = mu/rho), each evaluated with one rounding per operation and IEEE
// division / square root, so the result does not depend on the reduction
// order.  The minima are exact: positive doubles order like their bit
// patterns, so a 64-bit unsigned atomic min over the bits is exact and
// order independent.  dt = cfl * min(visc / alpha_v, conv).
#pragma once
#include "meg7_device.hpp"

namespace gbr {

struct DtParams {
  const double* __restrict__ Q;
  unsigned long long* mins;  // [2]: conv, visc (bit patterns)
  double* dt;
  unsigned* status;
  int nx, ny;
  double dx, dy, gamma, mu, cfl;
};

__global__ void dt_init_kernel(unsigned long long* mins) {
  if (threadIdx.x < 2) mins[threadIdx.x] = 0x7ff0000000000000ull;  // +inf
}

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long w = __shfl_xor(v, o);
    v = w < v ? w : v;
  }
  return v;
}

__global__ __launch_bounds__(256) void dt_reduce_kernel(DtParams P) {
#pragma clang fp contract(off)
  const size_t n = (size_t)P.nx * P.ny;
  double conv = __builtin_inf(), visc = __builtin_inf();
  bool bad = false;
  for (size_t s = (size_t)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (size_t)gridDim.x * blockDim.x) {
    const double rho = P.Q[s];
    const double u = P.Q[n + s] / rho, v = P.Q[2 * n + s] / rho;
    const double p = (P.gamma - 1.0) * (P.Q[3 * n + s] - rho * (u * u + v * v) / 2.0);
    const double c = sqrt(P.gamma * p / rho);
    // fmin drops NaN, so a bad cell is recorded explicitly
    if (!(rho > 0.0) || !(p > 0.0) || !isfinite(c) || !isfinite(u) || !isfinite(v)) bad = true;
    conv = fmin(conv, fmin(P.dx / (fabs(u) + c), P.dy / (fabs(v) + c)));
    if (P.mu > 0.0) {
      const double nu = P.mu / rho;
      visc = fmin(visc, fmin(P.dx * P.dx / nu, P.dy * P.dy / nu));
    }
  }
  if (bad) atomicOr(P.status, 1u);
  unsigned long long bc = __double_as_longlong(conv), bv = __double_as_longlong(visc);
  // a NaN (bad state) must not be hidden by the min: map it to the smallest key
  if (conv != conv) bc = 0ull;
  if (visc != visc) bv = 0ull;
  bc = wave_min_u64(bc);
  bv = wave_min_u64(bv);
  if (__lane_id() == 0) {
    atomicMin(&P.mins[0], bc);
    atomicMin(&P.mins[1], bv);
  }
}

__global__ void dt_finish_kernel(const unsigned long long* mins, double* dt, double cfl,
                                 unsigned* status) {
#pragma clang fp contract(off)
  if (threadIdx.x == 0) {
    const double conv = __longlong_as_double(mins[0]);
    const double visc = __longlong_as_double(mins[1]);
    const double d = cfl * fmin(visc / kAlphaV, conv);
    *dt = d;
    if (!(d > 0.0) || !isfinite(d)) atomicOr(status, 2u);
  }
}

}  // namespace gbr
