// C ABI of the MEG7 hot path (declared in include/gbr.h): context, argument
// checks, launches.  Every entry point validates its arguments before
// enqueueing anything and maps HIP errors to GBR_EDEVICE.
#include <hip/hip_runtime.h>

#include <new>

#include "../../include/gbr.h"
#include "dt_kernel.hpp"
#include "stage_f32.hpp"
#include "stage_kernel.hpp"

namespace {

using namespace gbr;

template <class C>
void launch_cfg(const StageParams& P, hipStream_t s) {
  static_assert(C::LDS_BYTES <= 160 * 1024, "LDS per workgroup");
  hipLaunchKernelGGL(meg7_stage_kernel<C>, dim3(P.ntiles), dim3(C::NT), 0, s, P);
}
template <class C>
void launch_cfg_f32(const StageParams& P, hipStream_t s) {
  static_assert(F32Cfg<C>::LDS_BYTES <= 160 * 1024, "LDS per workgroup");
  hipLaunchKernelGGL(meg7_stage_kernel_f32<C>, dim3(P.ntiles), dim3(C::NT), 0, s, P);
}
using LaunchFn = void (*)(const StageParams&, hipStream_t);

// Tile shapes of the stage kernel: TX x TY cells per workgroup, x sweep in
// sub-blocks of SX rows, y sweep in sub-blocks of SY columns, 256 threads.
// Shapes trade halo recomputation (small tiles) against LDS per workgroup
// (workgroups per CU); gbr_autotune times them on the caller's state.
struct TileVariant {
  int tx, ty;
  LaunchFn euler, visc;       // FP64; null: no build for this shape (use variant 0)
  LaunchFn euler32, visc32;   // FP32 bulk
  const char* name;
};
const TileVariant kVariants[] = {
    // 32 x-interfaces per row, 16 y-interfaces per column; 2 workgroups/CU
    {31, 15, launch_cfg<TileCfg<31, 15, 15, 16, 256, false>>,
     launch_cfg<TileCfg<31, 15, 8, 16, 256, true>>,
     launch_cfg_f32<TileCfg<31, 15, 15, 16, 256, false>>,
     launch_cfg_f32<TileCfg<31, 15, 8, 16, 256, true>>, "31x15"},
    // 16 interfaces per line both ways; 3 (Euler) / 2 (viscous) workgroups/CU
    {15, 15, launch_cfg<TileCfg<15, 15, 15, 15, 256, false>>,
     launch_cfg<TileCfg<15, 15, 15, 15, 256, true>>,
     launch_cfg_f32<TileCfg<15, 15, 15, 15, 256, false>>,
     launch_cfg_f32<TileCfg<15, 15, 15, 15, 256, true>>, "15x15"},
    // 64 x-interfaces per row, 8 y-interfaces per column (Euler only)
    {63, 7, launch_cfg<TileCfg<63, 7, 7, 32, 256, false>>, nullptr,
     launch_cfg_f32<TileCfg<63, 7, 7, 32, 256, false>>, nullptr, "63x7"},
    // 31x8 / 15x16 interface blocks sized for 3 workgroups per CU in FP32 bulk
    {30, 15, launch_cfg<TileCfg<30, 15, 15, 15, 256, false>>, nullptr,
     launch_cfg_f32<TileCfg<30, 15, 8, 15, 256, false, 3>>, nullptr, "30x15"},
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

}  // namespace

struct gbr_ctx {
  int nx, ny;
  double gamma, mu, Pr;
  double x0, x1, y0, y1;
  int bcx, bcy;
  int recon, mp_mode, precision, detector;
  int device;
  int export_flags;
  unsigned* d_status;         // [4]
  double* d_partial;          // [2][kDtBlocks] time-step partial minima
  uint8_t* d_sigx;
  uint8_t* d_sigy;
  int tiling;                 // index into kVariants
};

extern "C" {

const char* gbr_strerror(int s) {
  switch (s) {
    case GBR_OK: return "ok";
    case GBR_EINVAL: return "invalid argument";
    case GBR_ENOMEM: return "device allocation failed";
    case GBR_EDEVICE: return "HIP runtime error";
    case GBR_ESTATE: return "non-finite value or non-positive density/pressure on the device";
    case GBR_EUNSUPPORTED: return "option not supported by this build";
    default: return "unknown status";
  }
}

const char* gbr_version(void) { return "gbr-mi355x 0.2 (gfx950, MEG7-prim FP64 / FP32-bulk)"; }

static int hip_ok(hipError_t e) { return e == hipSuccess ? GBR_OK : GBR_EDEVICE; }

int gbr_init(int nx, int ny, double gamma, double mu, double Pr, gbr_ctx** out) {
  if (!out) return GBR_EINVAL;
  *out = nullptr;
  if (nx < 12 || ny < 12 || !(gamma > 1.0) || !(mu >= 0.0) || !(Pr > 0.0)) return GBR_EINVAL;
  if ((long long)nx * ny > (1ll << 31) / 4) return GBR_EINVAL;
  gbr_ctx* c = new (std::nothrow) gbr_ctx();
  if (!c) return GBR_ENOMEM;
  c->nx = nx; c->ny = ny; c->gamma = gamma; c->mu = mu; c->Pr = Pr;
  c->x0 = 0.0; c->x1 = 1.0; c->y0 = 0.0; c->y1 = 1.0;
  c->bcx = c->bcy = GBR_BC_PERIODIC;
  c->recon = GBR_RECON_PRIM; c->mp_mode = GBR_MP_FLAGGED;
  c->precision = GBR_PREC_FP64; c->detector = GBR_DET_PLAIN;
  if (hipGetDevice(&c->device) != hipSuccess) { delete c; return GBR_EDEVICE; }
  if (hipMalloc(&c->d_status, 4 * sizeof(unsigned)) != hipSuccess) { delete c; return GBR_ENOMEM; }
  if (hipMalloc(&c->d_partial, 2 * kDtBlocks * sizeof(double)) != hipSuccess) {
    (void)hipFree(c->d_status); delete c; return GBR_ENOMEM;
  }
  if (hipMemset(c->d_status, 0, 4 * sizeof(unsigned)) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    (void)hipFree(c->d_status); (void)hipFree(c->d_partial); delete c; return GBR_EDEVICE;
  }
  *out = c;
  return GBR_OK;
}

int gbr_destroy(gbr_ctx* c) {
  if (!c) return GBR_OK;
  (void)hipDeviceSynchronize();
  (void)hipFree(c->d_status);
  (void)hipFree(c->d_partial);
  if (c->d_sigx) (void)hipFree(c->d_sigx);
  if (c->d_sigy) (void)hipFree(c->d_sigy);
  delete c;
  return GBR_OK;
}

int gbr_set_geometry(gbr_ctx* c, double x0, double x1, double y0, double y1, int bc_x,
                     int bc_y) {
  if (!c || !(x1 > x0) || !(y1 > y0)) return GBR_EINVAL;
  if ((bc_x != GBR_BC_PERIODIC && bc_x != GBR_BC_TRANSMISSIVE) ||
      (bc_y != GBR_BC_PERIODIC && bc_y != GBR_BC_TRANSMISSIVE))
    return GBR_EINVAL;
  c->x0 = x0; c->x1 = x1; c->y0 = y0; c->y1 = y1; c->bcx = bc_x; c->bcy = bc_y;
  return GBR_OK;
}

int gbr_set_scheme(gbr_ctx* c, int recon, int mp_mode, int precision, int detector) {
  if (!c) return GBR_EINVAL;
  if (recon != GBR_RECON_PRIM || mp_mode != GBR_MP_FLAGGED) return GBR_EUNSUPPORTED;
  if (precision != GBR_PREC_FP64 && precision != GBR_PREC_FP32_BULK) return GBR_EUNSUPPORTED;
  if (detector != GBR_DET_PLAIN) return GBR_EUNSUPPORTED;
  c->recon = recon; c->mp_mode = mp_mode; c->precision = precision; c->detector = detector;
  return GBR_OK;
}

int gbr_export_flags(gbr_ctx* c, int enable) {
  if (!c) return GBR_EINVAL;
  if (enable && !c->d_sigx) {
    if (hipMalloc(&c->d_sigx, (size_t)c->ny * (c->nx + 1)) != hipSuccess) return GBR_ENOMEM;
    if (hipMalloc(&c->d_sigy, (size_t)(c->ny + 1) * c->nx) != hipSuccess) {
      (void)hipFree(c->d_sigx); c->d_sigx = nullptr; return GBR_ENOMEM;
    }
  }
  c->export_flags = enable ? 1 : 0;
  return GBR_OK;
}

int gbr_get_flags(gbr_ctx* c, uint8_t* sig_x, uint8_t* sig_y, void* stream) {
  if (!c || !c->d_sigx) return GBR_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (sig_x && hipMemcpyAsync(sig_x, c->d_sigx, (size_t)c->ny * (c->nx + 1), hipMemcpyDefault,
                              s) != hipSuccess)
    return GBR_EDEVICE;
  if (sig_y && hipMemcpyAsync(sig_y, c->d_sigy, (size_t)(c->ny + 1) * c->nx, hipMemcpyDefault,
                              s) != hipSuccess)
    return GBR_EDEVICE;
  return hip_ok(hipStreamSynchronize(s));
}

int gbr_check(gbr_ctx* c, void* stream) {
  if (!c) return GBR_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  unsigned h[4] = {0, 0, 0, 0};
  if (hipStreamSynchronize(s) != hipSuccess) return GBR_EDEVICE;
  if (hipMemcpy(h, c->d_status, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess)
    return GBR_EDEVICE;
  if (hipMemset(c->d_status, 0, sizeof(h)) != hipSuccess) return GBR_EDEVICE;
  if (hipDeviceSynchronize() != hipSuccess) return GBR_EDEVICE;
  return (h[0] | h[1] | h[2] | h[3]) ? GBR_ESTATE : GBR_OK;
}

static int launch_stage(gbr_ctx* c, int mode, const double* dt, const double* Qn,
                        const double* Qk, double* out, hipStream_t s) {
  StageParams P{};
  P.Qk = Qk; P.Qn = Qn; P.out = out; P.dt = dt;
  P.sigx = c->export_flags ? c->d_sigx : nullptr;
  P.sigy = c->export_flags ? c->d_sigy : nullptr;
  P.status = c->d_status;
  P.nx = c->nx; P.ny = c->ny; P.bcx = c->bcx; P.bcy = c->bcy;
  P.inv_dx = (double)c->nx / (c->x1 - c->x0);
  P.inv_dy = (double)c->ny / (c->y1 - c->y0);
  P.gamma = c->gamma; P.g1inv = 1.0 / (c->gamma - 1.0); P.mu = c->mu;
  P.kq = c->mu / (c->Pr * (c->gamma - 1.0));
  P.mode = mode;
  const bool visc = c->mu > 0.0;
  const TileVariant* v = &kVariants[c->tiling];
  if (visc && !v->visc) v = &kVariants[0];
  P.tiles_x = (c->nx + v->tx - 1) / v->tx;
  P.ntiles = P.tiles_x * ((c->ny + v->ty - 1) / v->ty);
  LaunchFn fn = (c->precision == GBR_PREC_FP32_BULK) ? (visc ? v->visc32 : v->euler32)
                                                       : (visc ? v->visc : v->euler);
  fn(P, s);
  return hip_ok(hipGetLastError());
}

int gbr_tiling_count(void) { return kNumVariants; }

int gbr_set_tiling(gbr_ctx* c, int variant) {
  if (!c || variant < 0 || variant >= kNumVariants) return GBR_EINVAL;
  c->tiling = variant;
  return GBR_OK;
}

int gbr_get_tiling(gbr_ctx* c, int* variant, int* tile_x, int* tile_y) {
  if (!c) return GBR_EINVAL;
  const TileVariant* v = &kVariants[c->tiling];
  if (c->mu > 0.0 && !v->visc) v = &kVariants[0];
  if (variant) *variant = (int)(v - kVariants);
  if (tile_x) *tile_x = v->tx;
  if (tile_y) *tile_y = v->ty;
  return GBR_OK;
}

int gbr_autotune(gbr_ctx* c, const double* Q, int reps, void* stream) {
  if (!c || !Q || reps < 1) return GBR_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  double* tmp = nullptr;
  if (hipMalloc(&tmp, sizeof(double) * 4 * (size_t)c->nx * c->ny) != hipSuccess) return GBR_ENOMEM;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    (void)hipFree(tmp);
    return GBR_EDEVICE;
  }
  const int saved = c->tiling, flags = c->export_flags;
  c->export_flags = 0;
  int best = saved, rc = GBR_OK;
  float best_ms = 1e30f;
  for (int v = 0; v < kNumVariants && rc == GBR_OK; ++v) {
    if (c->mu > 0.0 && !kVariants[v].visc) continue;
    c->tiling = v;
    rc = launch_stage(c, MODE_RESIDUAL, nullptr, Q, Q, tmp, s);  // warm-up
    if (rc != GBR_OK) break;
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps && rc == GBR_OK; ++r) rc = launch_stage(c, MODE_RESIDUAL, nullptr, Q, Q, tmp, s);
    (void)hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess) { rc = GBR_EDEVICE; break; }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms < best_ms) { best_ms = ms; best = v; }
  }
  c->tiling = (rc == GBR_OK) ? best : saved;
  c->export_flags = flags;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(tmp);
  return rc;
}

int gbr_residual(gbr_ctx* c, const double* Q, double* Res, void* stream) {
  if (!c || !Q || !Res || Q == Res) return GBR_EINVAL;
  return launch_stage(c, MODE_RESIDUAL, nullptr, Q, Q, Res, (hipStream_t)stream);
}

int gbr_rk_stage(gbr_ctx* c, int stage, const double* dt_dev, const double* Qn,
                 const double* Qk, double* Qout, void* stream) {
  if (!c || !dt_dev || !Qn || !Qk || !Qout) return GBR_EINVAL;
  if (stage < 1 || stage > 3) return GBR_EINVAL;
  if (Qout == Qn || Qout == Qk) return GBR_EINVAL;
  if (stage == 1 && Qk != Qn) return GBR_EINVAL;
  return launch_stage(c, stage, dt_dev, Qn, Qk, Qout, (hipStream_t)stream);
}

int gbr_compute_dt(gbr_ctx* c, const double* Q, double cfl, double* dt_dev, void* stream) {
  if (!c || !Q || !dt_dev || !(cfl > 0.0)) return GBR_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  DtParams P{};
  P.Q = Q; P.partial = c->d_partial; P.dt = dt_dev; P.status = c->d_status;
  P.nx = c->nx; P.ny = c->ny;
  P.dx = (c->x1 - c->x0) / c->nx; P.dy = (c->y1 - c->y0) / c->ny;
  P.gamma = c->gamma; P.mu = c->mu; P.cfl = cfl;
  const size_t n = (size_t)c->nx * c->ny;
  size_t want = (n + kDtThreads - 1) / kDtThreads;
  const int blocks = (int)(want < (size_t)kDtBlocks ? want : (size_t)kDtBlocks);
  hipLaunchKernelGGL(dt_reduce_kernel, dim3(blocks), dim3(kDtThreads), 0, s, P);
  hipLaunchKernelGGL(dt_finish_kernel, dim3(1), dim3(kDtThreads), 0, s, c->d_partial, blocks,
                     dt_dev, cfl, c->d_status);
  return hip_ok(hipGetLastError());
}

}  // extern "C"
