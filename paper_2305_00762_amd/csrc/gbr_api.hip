// C ABI of the MEG7 hot path (declared in include/gbr.h): context, argument
// checks, launches.  Every entry point validates its arguments before
// enqueueing anything and maps HIP errors to GBR_EDEVICE.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/gbr.h"
#include "batch_kernel.hpp"
#include "dt_kernel.hpp"
#include "mlp_kernels.hpp"
#include "stage3d.hpp"
#include "stage_f32.hpp"
#include "stage_kernel.hpp"

namespace {

using namespace gbr;

// Threads per workgroup of every single-grid stage kernel: a stage-3 launch
// leaves one time-step slot per wave, kStageThreads / 64 per tile.
constexpr int kStageThreads = 256;
constexpr int kStageWaves = kStageThreads / 64;

template <class C, bool MLP = false, bool CONS = false, int ORD = 7, bool LM = false,
          bool MPE = false>
void launch_cfg(const StageParams& P, hipStream_t s) {
  static_assert(C::LDS_BYTES <= 160 * 1024, "LDS per workgroup");
  static_assert(C::NT == kStageThreads, "time-step slots assume kStageThreads per workgroup");
  hipLaunchKernelGGL((meg7_stage_kernel<C, MLP, CONS, ORD, LM, MPE>), dim3(P.ntiles), dim3(C::NT),
                     0, s, P);
}
template <class C, bool MLP = false>
void launch_cfg_f32(const StageParams& P, hipStream_t s) {
  static_assert(F32Cfg<C>::LDS_BYTES <= 160 * 1024, "LDS per workgroup");
  static_assert(C::NT == kStageThreads, "time-step slots assume kStageThreads per workgroup");
  hipLaunchKernelGGL((meg7_stage_kernel_f32<C, MLP>), dim3(P.ntiles), dim3(C::NT), 0, s, P);
}
using LaunchFn = void (*)(const StageParams&, hipStream_t);

// Tile shapes of the stage kernel: TX x TY cells per workgroup, x sweep in
// sub-blocks of SX rows, y sweep in sub-blocks of SY columns, 256 threads.
// Shapes trade halo recomputation (small tiles) against LDS per workgroup
// (workgroups per CU); gbr_autotune times them on the caller's state.
struct TileVariant {
  int tx, ty;
  LaunchFn fn[2][2][2];   // [precision FP64/FP32-bulk][viscous][learned detector]; null: no build
  const char* name;
  LaunchFn cons[2];       // MEG7-cons, FP64 with the plain detector: [viscous]; null: no build
  LaunchFn g4[2][2];      // fourth-order GRB, FP64 with the plain detector: [cons][viscous]
  LaunchFn ss[2][2];      // shock-stable HLLC, seventh order, FP64, plain: [cons][viscous]
  LaunchFn mpe[2][2];     // MP test at every interface, seventh order, FP64, plain: [cons][viscous]
};
using E31 = TileCfg<31, 15, 15, 16, 256, false>;
using V31 = TileCfg<31, 15, 8, 16, 256, true>;
// FP64 on 15x15 tiles: 3 workgroups per CU fit the LDS, so the register
// budget is held to 3 waves per SIMD (168 VGPRs)
using E15 = TileCfg<15, 15, 15, 15, 256, false, 3>;
using V15 = TileCfg<15, 15, 15, 15, 256, true, 3>;
// FP32 bulk on 15x15 tiles: 4 workgroups per CU fit the LDS, so the register
// budget is held to 4 waves per SIMD (128 VGPRs)
using F15 = TileCfg<15, 15, 15, 15, 256, false, 4>;
using FV15 = TileCfg<15, 15, 15, 15, 256, true, 4>;
const TileVariant kVariants[] = {
    // 32 x-interfaces per row, 16 y-interfaces per column; 2 workgroups/CU
    {31, 15,
     {{{launch_cfg<E31>, launch_cfg<E31, true>}, {launch_cfg<V31>, launch_cfg<V31, true>}},
      {{launch_cfg_f32<E31>, launch_cfg_f32<E31, true>},
       {launch_cfg_f32<V31>, launch_cfg_f32<V31, true>}}},
     "31x15",
     {launch_cfg<E31, false, true>, launch_cfg<V31, false, true>},
     {{launch_cfg<E31, false, false, 4>, launch_cfg<V31, false, false, 4>},
      {launch_cfg<E31, false, true, 4>, launch_cfg<V31, false, true, 4>}},
     {{launch_cfg<E31, false, false, 7, true>, launch_cfg<V31, false, false, 7, true>},
      {launch_cfg<E31, false, true, 7, true>, launch_cfg<V31, false, true, 7, true>}},
     {{launch_cfg<E31, false, false, 7, false, true>, launch_cfg<V31, false, false, 7, false, true>},
      {launch_cfg<E31, false, true, 7, false, true>, launch_cfg<V31, false, true, 7, false, true>}}},
    // 16 interfaces per line both ways; 3-4 workgroups/CU
    {15, 15,
     {{{launch_cfg<E15>, launch_cfg<E15, true>}, {launch_cfg<V15>, launch_cfg<V15, true>}},
      {{launch_cfg_f32<F15>, launch_cfg_f32<F15, true>},
       {launch_cfg_f32<FV15>, launch_cfg_f32<FV15, true>}}},
     "15x15",
     {launch_cfg<E15, false, true>, launch_cfg<V15, false, true>},
     {{launch_cfg<E15, false, false, 4>, launch_cfg<V15, false, false, 4>},
      {launch_cfg<E15, false, true, 4>, launch_cfg<V15, false, true, 4>}},
     {{launch_cfg<E15, false, false, 7, true>, launch_cfg<V15, false, false, 7, true>},
      {launch_cfg<E15, false, true, 7, true>, launch_cfg<V15, false, true, 7, true>}},
     {{launch_cfg<E15, false, false, 7, false, true>, launch_cfg<V15, false, false, 7, false, true>},
      {launch_cfg<E15, false, true, 7, false, true>, launch_cfg<V15, false, true, 7, false, true>}}},
    // 64 x-interfaces per row, 8 y-interfaces per column (Euler, plain detector)
    {63, 7,
     {{{launch_cfg<TileCfg<63, 7, 7, 32, 256, false>>,
        launch_cfg<TileCfg<63, 7, 7, 32, 256, false>, true>},
       {nullptr, nullptr}},
      {{launch_cfg_f32<TileCfg<63, 7, 7, 32, 256, false>>,
        launch_cfg_f32<TileCfg<63, 7, 7, 32, 256, false>, true>},
       {nullptr, nullptr}}},
     "63x7",
     {nullptr, nullptr},
     {{nullptr, nullptr}, {nullptr, nullptr}},
     {{nullptr, nullptr}, {nullptr, nullptr}},
     {{nullptr, nullptr}, {nullptr, nullptr}}},
    // 31x8 / 15x16 interface blocks sized for 3 workgroups per CU in FP32 bulk
    {30, 15,
     {{{launch_cfg<TileCfg<30, 15, 15, 15, 256, false>>,
        launch_cfg<TileCfg<30, 15, 15, 15, 256, false>, true>},
       {nullptr, nullptr}},
      {{launch_cfg_f32<TileCfg<30, 15, 8, 15, 256, false, 3>>,
        launch_cfg_f32<TileCfg<30, 15, 8, 15, 256, false, 3>, true>},
       {nullptr, nullptr}}},
     "30x15",
     {nullptr, nullptr},
     {{nullptr, nullptr}, {nullptr, nullptr}},
     {{nullptr, nullptr}, {nullptr, nullptr}},
     {{nullptr, nullptr}, {nullptr, nullptr}}},
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

// Forms of the batched kernel: tile shape (inviscid and viscous forms of one
// shape) x persistent tile loop or one workgroup per tile.
template <class CI, class CV, bool F32, int MW, bool LOOP>
void launch_batch(const BatchParams& B, int grid, hipStream_t s) {
  static_assert(BatchCfg<CI, CV, F32, MW>::LDS_BYTES <= 160 * 1024, "LDS per workgroup");
  hipLaunchKernelGGL((meg7_batch_kernel<CI, CV, F32, MW, LOOP>), dim3(grid), dim3(CI::NT), 0, s, B);
}
template <class CI, class CV, bool F32, int MW, bool LOOP>
int batch_blocks_per_cu() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, meg7_batch_kernel<CI, CV, F32, MW, LOOP>,
                                                    CI::NT, 0) != hipSuccess)
    return 0;
  return n;
}
using BatchLaunchFn = void (*)(const BatchParams&, int, hipStream_t);
struct BatchVariant {
  int tx, ty, loop;
  BatchLaunchFn fn[2];   // [FP64, FP32 bulk]
  int (*occ[2])();
  const char* name;
};
#define GBR_BATCH_VARIANT(TX, TY, CI, CV, MW64, MW32, LOOP, NAME)                     \
  {TX, TY, LOOP,                                                                      \
   {launch_batch<CI, CV, false, MW64, LOOP>, launch_batch<CI, CV, true, MW32, LOOP>}, \
   {batch_blocks_per_cu<CI, CV, false, MW64, LOOP>,                                   \
    batch_blocks_per_cu<CI, CV, true, MW32, LOOP>},                                   \
   NAME}
const BatchVariant kBatchVariants[] = {
    GBR_BATCH_VARIANT(31, 15, E31, V31, 2, 2, true, "31x15 persistent"),
    GBR_BATCH_VARIANT(15, 15, E15, V15, 3, 2, true, "15x15 persistent"),
    GBR_BATCH_VARIANT(31, 15, E31, V31, 2, 2, false, "31x15 one tile per workgroup"),
    GBR_BATCH_VARIANT(15, 15, E15, V15, 2, 4, false, "15x15 one tile per workgroup"),
};
#undef GBR_BATCH_VARIANT
constexpr int kNumBatchVariants = sizeof(kBatchVariants) / sizeof(kBatchVariants[0]);

}  // namespace

struct gbr_ctx {
  int nx, ny;
  double gamma, mu, Pr;
  double x0, x1, y0, y1;
  int bcx, bcy;
  int recon, mp_mode, precision, detector;
  int order;                  // GRB order: 7 or 4
  int riemann;                // 0: HLLC, 1: shock-stable HLLC
  int use_sides;              // 1: the side table d_sides replaces bcx / bcy
  SideDev* d_sides;           // [4] left, right, bottom, top
  double* d_time;             // device time of Q^n (moving boundary segments)
  int device;
  int export_flags;
  unsigned* d_status;         // [4]
  double* d_partial;          // [3][kDtBlocks] time-step partial extrema
  double* d_dtx;              // [3][slots] per-wave time-step extrema of a stage-3 output
  int dtx_cap;                // slots d_dtx holds (the most of any tile shape)
  int stage3_slots;           // slots of the last stage-3 call; 0: none since gbr_stage_dt
  uint8_t* d_sigx;
  uint8_t* d_sigy;
  int tiling;                 // index into kVariants
  // learned detector: inference image (bf16 W1, W2; float w3, biases)
  unsigned short* d_mlp_w;    // [2][32][32]
  float* d_mlp_f;             // [32 + 65]
  float mlp_margin;
  int mlp_ready;
  uint8_t* d_chimap;          // [ny][nx] learned-detector flag per cell
  int mlp_reuse;              // 1: flag map evaluated on Q^n only (residual and stage 1)
  int chimap_valid;           // a flag map has been evaluated
  // per-step detector: float32 (rho, p) of the last stage-3 output [2][ny][nx],
  // written by that stage kernel and read by the next flag map in place of Q
  // when gbr_stage_dt took the step's time step from that output (armed)
  float* d_rp;
  const double* rp_src;       // the stage-3 output d_rp describes
  int rp_valid;
  int rp_armed;
  unsigned long long* d_mlp_fb;   // plain fallbacks of the learned detector
  unsigned long long mlp_evaluated;
  // kernel timing (gbr_timing): events recorded around every launch of a
  // residual or stage call, three per call: before the learned detector's
  // flag map, before the stage kernel, after it
  int timing;
  std::vector<hipEvent_t> ev;
  size_t ev_used;
};

struct gbr_mlp {
  int device;
  float* d_master;            // [kMlpNP] float32 parameters (weights, then biases)
  float* d_m;                 // Adam moments
  float* d_v;
  unsigned short* d_w;        // bf16 inference image [2][32][32]
  float* d_f;                 // [32 + 65]
  float* d_partial;           // [kMlpMaxBlocks][kMlpNP + 1]
  float* d_grad;              // [kMlpNP + 1]
  int t;                      // Adam step count
};

// Scratch of the entry point that allocates nothing (gbr_compute_dt_noalloc):
// the first pass's partial minima [2][kDtBlocks], then a status word.  In host
// code the name `scratch` is only a stand-in for the device array: its device
// address, one per GPU, comes from hipGetSymbolAddress and is kept below.
constexpr int kNoallocScratchDoubles = 2 * gbr::kDtBlocks + 32;
static __device__ __align__(256) double scratch[kNoallocScratchDoubles];
constexpr int kNoallocMaxDevices = 64;
static std::mutex g_scratch_mutex;
static double* g_scratch_ptr[kNoallocMaxDevices];

// Device address of `scratch` on the current device, looked up once per
// device with that device current.
static int noalloc_scratch(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return GBR_EDEVICE;
  if (dev < 0 || dev >= kNoallocMaxDevices) return GBR_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GBR_EDEVICE;
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return GBR_OK;
}

extern "C" {

const char* gbr_strerror(int s) {
  switch (s) {
    case GBR_OK: return "ok";
    case GBR_EINVAL: return "invalid argument";
    case GBR_ENOMEM: return "device allocation failed";
    case GBR_EDEVICE: return "HIP runtime error";
    case GBR_ESTATE: return "non-finite value or non-positive density/pressure on the device";
    case GBR_EUNSUPPORTED: return "option not supported by the library";
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
  c->recon = GBR_RECON_PRIM; c->mp_mode = GBR_MP_FLAGGED; c->order = 7;
  c->precision = GBR_PREC_FP64; c->detector = GBR_DET_PLAIN;
  if (hipGetDevice(&c->device) != hipSuccess) { delete c; return GBR_EDEVICE; }
  if (hipMalloc(&c->d_status, 4 * sizeof(unsigned)) != hipSuccess) { delete c; return GBR_ENOMEM; }
  if (hipMalloc(&c->d_partial, 3 * kDtBlocks * sizeof(double)) != hipSuccess) {
    (void)hipFree(c->d_status); delete c; return GBR_ENOMEM;
  }
  if (hipMalloc(&c->d_sides, 4 * sizeof(SideDev)) != hipSuccess) {
    (void)hipFree(c->d_status); (void)hipFree(c->d_partial); delete c; return GBR_ENOMEM;
  }
  if (hipMalloc(&c->d_time, sizeof(double)) != hipSuccess) {
    (void)hipFree(c->d_status); (void)hipFree(c->d_partial); (void)hipFree(c->d_sides);
    delete c; return GBR_ENOMEM;
  }
  // per-wave time-step extrema of stage-3 outputs: room for the waves of
  // the smallest tile shape
  c->dtx_cap = 0;
  for (int v = 0; v < kNumVariants; ++v) {
    const int t = ((nx + kVariants[v].tx - 1) / kVariants[v].tx) *
                  ((ny + kVariants[v].ty - 1) / kVariants[v].ty) * kStageWaves;
    c->dtx_cap = t > c->dtx_cap ? t : c->dtx_cap;
  }
  if (hipMalloc(&c->d_dtx, 3 * (size_t)c->dtx_cap * sizeof(double)) != hipSuccess) {
    (void)hipFree(c->d_status); (void)hipFree(c->d_partial); (void)hipFree(c->d_sides);
    (void)hipFree(c->d_time); delete c; return GBR_ENOMEM;
  }
  double* noalloc = nullptr;   // set-up of the allocation-free entry point on this device
  if (hipMemset(c->d_status, 0, 4 * sizeof(unsigned)) != hipSuccess ||
      hipMemset(c->d_time, 0, sizeof(double)) != hipSuccess ||
      noalloc_scratch(&noalloc) != GBR_OK || hipDeviceSynchronize() != hipSuccess) {
    (void)hipFree(c->d_status); (void)hipFree(c->d_partial); (void)hipFree(c->d_sides);
    (void)hipFree(c->d_time); (void)hipFree(c->d_dtx); delete c; return GBR_EDEVICE;
  }
  *out = c;
  return GBR_OK;
}

int gbr_destroy(gbr_ctx* c) {
  if (!c) return GBR_OK;
  (void)hipDeviceSynchronize();
  (void)hipFree(c->d_status);
  (void)hipFree(c->d_partial);
  (void)hipFree(c->d_sides);
  (void)hipFree(c->d_time);
  (void)hipFree(c->d_dtx);
  if (c->d_sigx) (void)hipFree(c->d_sigx);
  if (c->d_sigy) (void)hipFree(c->d_sigy);
  if (c->d_mlp_w) (void)hipFree(c->d_mlp_w);
  if (c->d_mlp_f) (void)hipFree(c->d_mlp_f);
  if (c->d_chimap) (void)hipFree(c->d_chimap);
  if (c->d_mlp_fb) (void)hipFree(c->d_mlp_fb);
  if (c->d_rp) (void)hipFree(c->d_rp);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
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
  c->use_sides = 0;
  return GBR_OK;
}

int gbr_set_sides(gbr_ctx* c, const gbr_side* sides) {
  if (!c) return GBR_EINVAL;
  if (!sides) { c->use_sides = 0; return GBR_OK; }
  for (int a = 0; a < 2; ++a) {
    int nper = 0;
    for (int sd = 2 * a; sd < 2 * a + 2; ++sd)
      for (int g = 0; g < 2; ++g) {
        const int k = sides[sd].kind[g];
        if (k < GBR_BC_PERIODIC || k > GBR_BC_INFLOW) return GBR_EINVAL;
        nper += (k == GBR_BC_PERIODIC);
        if (k == GBR_BC_INFLOW) {
          const double* st = sides[sd].state[g];
          if (!(st[0] > 0.0) || !(st[3] > 0.0) || !std::isfinite(st[1]) || !std::isfinite(st[2]) ||
              !std::isfinite(st[0]) || !std::isfinite(st[3]))
            return GBR_EINVAL;
        }
      }
    if (nper != 0 && nper != 4) return GBR_EINVAL;
    for (int sd = 2 * a; sd < 2 * a + 2; ++sd)
      if (std::isnan(sides[sd].split0) || !std::isfinite(sides[sd].split_speed)) return GBR_EINVAL;
  }
  if (c->precision != GBR_PREC_FP64 || c->detector != GBR_DET_PLAIN) return GBR_EUNSUPPORTED;
  static_assert(sizeof(SideDev) == sizeof(gbr_side), "side layout");
  if (hipMemcpy(c->d_sides, sides, 4 * sizeof(SideDev), hipMemcpyHostToDevice) != hipSuccess)
    return GBR_EDEVICE;
  c->use_sides = 1;
  return GBR_OK;
}

int gbr_set_riemann(gbr_ctx* c, int kind) {
  if (!c || (kind != GBR_RIEMANN_HLLC && kind != GBR_RIEMANN_HLLC_SS)) return GBR_EINVAL;
  if (kind == GBR_RIEMANN_HLLC_SS &&
      (c->precision != GBR_PREC_FP64 || c->detector != GBR_DET_PLAIN || c->order != 7 ||
       c->mp_mode != GBR_MP_FLAGGED))
    return GBR_EUNSUPPORTED;
  c->riemann = kind;
  return GBR_OK;
}

int gbr_set_time(gbr_ctx* c, double t) {
  if (!c || !std::isfinite(t)) return GBR_EINVAL;
  if (hipMemcpy(c->d_time, &t, sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
    return GBR_EDEVICE;
  return GBR_OK;
}

int gbr_get_time(gbr_ctx* c, double* t) {
  if (!c || !t) return GBR_EINVAL;
  if (hipMemcpy(t, c->d_time, sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
    return GBR_EDEVICE;
  return GBR_OK;
}

int gbr_advance_time(gbr_ctx* c, const double* dt_dev, void* stream) {
  if (!c || !dt_dev) return GBR_EINVAL;
  hipLaunchKernelGGL(advance_time_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, c->d_time,
                     dt_dev);
  return hip_ok(hipGetLastError());
}

int gbr_set_scheme(gbr_ctx* c, int recon, int mp_mode, int precision, int detector) {
  if (!c) return GBR_EINVAL;
  if (recon != GBR_RECON_PRIM && recon != GBR_RECON_CONS) return GBR_EUNSUPPORTED;
  if (mp_mode != GBR_MP_FLAGGED && mp_mode != GBR_MP_EVERYWHERE) return GBR_EUNSUPPORTED;
  if (mp_mode == GBR_MP_EVERYWHERE &&
      (precision != GBR_PREC_FP64 || detector != GBR_DET_PLAIN || c->order != 7 ||
       c->riemann != GBR_RIEMANN_HLLC))
    return GBR_EUNSUPPORTED;
  if (precision != GBR_PREC_FP64 && precision != GBR_PREC_FP32_BULK) return GBR_EUNSUPPORTED;
  if (detector != GBR_DET_PLAIN && detector != GBR_DET_MLP) return GBR_EUNSUPPORTED;
  if ((recon == GBR_RECON_CONS || c->order == 4 || c->use_sides || c->riemann) &&
      (precision != GBR_PREC_FP64 || detector != GBR_DET_PLAIN))
    return GBR_EUNSUPPORTED;
  if (detector == GBR_DET_MLP && !c->mlp_ready) return GBR_EINVAL;
  c->recon = recon; c->mp_mode = mp_mode; c->precision = precision; c->detector = detector;
  return GBR_OK;
}

int gbr_set_order(gbr_ctx* c, int order) {
  if (!c) return GBR_EINVAL;
  if (order != 7 && order != 4) return GBR_EINVAL;
  if (order == 4 && (c->precision != GBR_PREC_FP64 || c->detector != GBR_DET_PLAIN ||
                     c->riemann != GBR_RIEMANN_HLLC || c->mp_mode != GBR_MP_FLAGGED))
    return GBR_EUNSUPPORTED;
  c->order = order;
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

// Launcher of tile variant v for the context's scheme, or null where the
// variant has no build for it.
static LaunchFn variant_fn(const gbr_ctx* c, int v) {
  const int visc = c->mu > 0.0 ? 1 : 0;
  if (c->mp_mode == GBR_MP_EVERYWHERE)
    return kVariants[v].mpe[c->recon == GBR_RECON_CONS ? 1 : 0][visc];
  if (c->riemann == GBR_RIEMANN_HLLC_SS)
    return kVariants[v].ss[c->recon == GBR_RECON_CONS ? 1 : 0][visc];
  if (c->order == 4) return kVariants[v].g4[c->recon == GBR_RECON_CONS ? 1 : 0][visc];
  if (c->recon == GBR_RECON_CONS) return kVariants[v].cons[visc];
  const int prec = c->precision == GBR_PREC_FP32_BULK ? 1 : 0;
  const int det = c->detector == GBR_DET_MLP ? 1 : 0;
  return kVariants[v].fn[prec][visc][det];
}
static int active_variant(const gbr_ctx* c) { return variant_fn(c, c->tiling) ? c->tiling : 0; }

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
  P.sides = c->use_sides ? c->d_sides : nullptr;
  P.tnow = c->d_time;
  // boundary time of stage k: t + c_k dt, c = (0, 1, 1/2)
  P.tc = mode == MODE_STAGE2 ? 1.0 : (mode == MODE_STAGE3 ? 0.5 : 0.0);
  P.x0 = c->x0; P.y0 = c->y0;
  P.dx = (c->x1 - c->x0) / c->nx; P.dy = (c->y1 - c->y0) / c->ny;
  P.dtx = mode == MODE_STAGE3 ? c->d_dtx : nullptr;
  const int det = c->detector == GBR_DET_MLP ? 1 : 0;
  // per-step detector: stages 2 and 3 reuse the flag map of Q^n, and stage 3
  // leaves (rho, p) of Q^(n+1) for the next step's flag map
  const bool reuse = det && c->mlp_reuse && (mode == MODE_STAGE2 || mode == MODE_STAGE3);
  if (reuse && !c->chimap_valid) return GBR_EINVAL;
  P.rp = (mode == MODE_STAGE3 && det && c->mlp_reuse) ? c->d_rp : nullptr;
  hipEvent_t* tev = nullptr;
  if (c->timing) {
    if (c->ev_used + 3 > c->ev.size()) {
      for (int k = 0; k < 3 * 64; ++k) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return GBR_EDEVICE;
        c->ev.push_back(e);
      }
    }
    tev = &c->ev[c->ev_used];
    c->ev_used += 3;
    if (hipEventRecord(tev[0], s) != hipSuccess) return GBR_EDEVICE;
  }
  if (det && !reuse) {
    MlpChiParams M{};
    M.Q = Qk; M.chi = c->d_chimap; M.nfb = c->d_mlp_fb;
    M.rp = (c->mlp_reuse && c->rp_armed && c->rp_valid && c->rp_src == Qk) ? c->d_rp : nullptr;
    c->rp_armed = 0;
    M.M.W1 = c->d_mlp_w;
    M.M.W2 = c->d_mlp_w + kMlpH * kMlpIn;
    M.M.w3 = c->d_mlp_f;
    M.M.b = c->d_mlp_f + kMlpH;
    M.margin = c->mlp_margin;
    M.nx = c->nx; M.ny = c->ny; M.bcx = c->bcx; M.bcy = c->bcy;
    M.tiles_x = (c->nx + kChiTX - 1) / kChiTX;
    M.gamma = c->gamma;
    const int nblk = M.tiles_x * ((c->ny + kChiTY - 1) / kChiTY);
    hipLaunchKernelGGL(mlp_chi_kernel, dim3(nblk), dim3(256), 0, s, M);
    c->mlp_evaluated += 2ull * c->nx * c->ny;   // along x and along y
    c->chimap_valid = 1;
  }
  if (det) P.chimap = c->d_chimap;
  const int vi = active_variant(c);
  const TileVariant* v = &kVariants[vi];
  P.tiles_x = (c->nx + v->tx - 1) / v->tx;
  P.ntiles = P.tiles_x * ((c->ny + v->ty - 1) / v->ty);
  if (tev && hipEventRecord(tev[1], s) != hipSuccess) return GBR_EDEVICE;
  variant_fn(c, vi)(P, s);
  if (tev && hipEventRecord(tev[2], s) != hipSuccess) return GBR_EDEVICE;
  if (mode == MODE_STAGE3) {
    c->stage3_slots = P.ntiles * kStageWaves;
    c->rp_valid = P.rp != nullptr;
    c->rp_src = out;
    c->rp_armed = 0;
  }
  return hip_ok(hipGetLastError());
}

int gbr_timing(gbr_ctx* c, int enable) {
  if (!c) return GBR_EINVAL;
  c->timing = enable ? 1 : 0;
  c->ev_used = 0;
  return GBR_OK;
}

int gbr_timing_read(gbr_ctx* c, double* detector_ms, double* stage_ms, uint64_t* launches) {
  if (!c) return GBR_EINVAL;
  double d = 0.0, st = 0.0;
  for (size_t k = 0; k + 3 <= c->ev_used; k += 3) {
    float a = 0.f, b = 0.f;
    if (hipEventSynchronize(c->ev[k + 2]) != hipSuccess ||
        hipEventElapsedTime(&a, c->ev[k], c->ev[k + 1]) != hipSuccess ||
        hipEventElapsedTime(&b, c->ev[k + 1], c->ev[k + 2]) != hipSuccess)
      return GBR_EDEVICE;
    d += a;
    st += b;
  }
  if (detector_ms) *detector_ms = d;
  if (stage_ms) *stage_ms = st;
  if (launches) *launches = c->ev_used / 3;
  c->ev_used = 0;
  return GBR_OK;
}

int gbr_tiling_count(void) { return kNumVariants; }

int gbr_set_tiling(gbr_ctx* c, int variant) {
  if (!c || variant < 0 || variant >= kNumVariants) return GBR_EINVAL;
  c->tiling = variant;
  return GBR_OK;
}

int gbr_get_tiling(gbr_ctx* c, int* variant, int* tile_x, int* tile_y) {
  if (!c) return GBR_EINVAL;
  const TileVariant* v = &kVariants[active_variant(c)];
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
  const int saved = c->tiling, flags = c->export_flags, timing = c->timing;
  c->export_flags = 0;
  c->timing = 0;
  int best = saved, rc = GBR_OK;
  float best_ms = 1e30f;
  for (int v = 0; v < kNumVariants && rc == GBR_OK; ++v) {
    if (!variant_fn(c, v)) continue;
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
  c->timing = timing;
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
  const int blocks = dt_blocks((size_t)c->nx * c->ny);
  hipLaunchKernelGGL(dt_reduce_kernel, dim3(blocks), dim3(kDtThreads), 0, s, P);
  hipLaunchKernelGGL(dt_finish_kernel, dim3(1), dim3(kDtThreads), 0, s, c->d_partial, blocks,
                     dt_dev, cfl, c->d_status);
  c->rp_armed = 0;   // a step begun from the state itself
  return hip_ok(hipGetLastError());
}

int gbr_compute_dt_noalloc(int nx, int ny, double dx, double dy, double gamma, double mu,
                           const double* Q, double cfl, double* dt_dev, void* stream) {
  if (nx < 1 || ny < 1 || (long long)nx * ny > (long long)GBR_NOALLOC_MAX_CELLS) return GBR_EINVAL;
  if (!Q || !dt_dev || !(dx > 0.0) || !(dy > 0.0) || !(gamma > 1.0) || !(mu >= 0.0) ||
      !(cfl > 0.0))
    return GBR_EINVAL;
  double* ptr = nullptr;
  const int rc = noalloc_scratch(&ptr);
  if (rc != GBR_OK) return rc;
  unsigned* status = reinterpret_cast<unsigned*>(ptr + 2 * kDtBlocks);
  hipStream_t s = (hipStream_t)stream;
  DtParams P{};
  P.Q = Q; P.partial = ptr; P.dt = dt_dev; P.status = status;
  P.nx = nx; P.ny = ny; P.dx = dx; P.dy = dy; P.gamma = gamma; P.mu = mu; P.cfl = cfl;
  const int blocks = dt_blocks((size_t)nx * ny);   // <= kDtBlocks: the partials fit
  hipLaunchKernelGGL(dt_reduce_kernel, dim3(blocks), dim3(kDtThreads), 0, s, P);
  hipLaunchKernelGGL(dt_finish_noalloc_kernel, dim3(1), dim3(kDtThreads), 0, s,
                     (const double*)ptr, blocks, dt_dev, cfl, status);
  return hip_ok(hipGetLastError());
}

int gbr_stage_dt(gbr_ctx* c, double cfl, double* dt_dev, void* stream) {
  if (!c || !dt_dev || !(cfl > 0.0) || c->stage3_slots <= 0) return GBR_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const int nslot = c->stage3_slots;
  const int blocks = dt_blocks((size_t)nslot);
  hipLaunchKernelGGL(dt_extrema_reduce_kernel<false>, dim3(blocks), dim3(kDtThreads), 0, s,
                     (const double*)c->d_dtx, nslot, c->d_partial);
  hipLaunchKernelGGL(dt_from_extrema_kernel, dim3(1), dim3(kDtThreads), 0, s,
                     (const double*)c->d_partial, blocks, dt_dev, cfl,
                     (c->x1 - c->x0) / c->nx, (c->y1 - c->y0) / c->ny, c->mu, c->d_status);
  c->stage3_slots = 0;
  c->rp_armed = c->rp_valid;
  return hip_ok(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Learned detector.
static constexpr int kMlpMaxBatch = 1 << 16;
static constexpr int kMlpMaxBlocks = kMlpMaxBatch / 256;

int gbr_mlp_create(gbr_mlp** out) {
  if (!out) return GBR_EINVAL;
  *out = nullptr;
  gbr_mlp* m = new (std::nothrow) gbr_mlp();
  if (!m) return GBR_ENOMEM;
  if (hipGetDevice(&m->device) != hipSuccess) { delete m; return GBR_EDEVICE; }
  bool ok = hipMalloc(&m->d_master, kMlpNP * sizeof(float)) == hipSuccess &&
            hipMalloc(&m->d_m, kMlpNP * sizeof(float)) == hipSuccess &&
            hipMalloc(&m->d_v, kMlpNP * sizeof(float)) == hipSuccess &&
            hipMalloc(&m->d_w, 2 * kMlpH * kMlpIn * sizeof(unsigned short)) == hipSuccess &&
            hipMalloc(&m->d_f, (kMlpH + kMlpNB) * sizeof(float)) == hipSuccess &&
            hipMalloc(&m->d_partial, (size_t)kMlpMaxBlocks * (kMlpNP + 1) * sizeof(float)) == hipSuccess &&
            hipMalloc(&m->d_grad, (kMlpNP + 1) * sizeof(float)) == hipSuccess;
  if (!ok) { gbr_mlp_destroy(m); return GBR_ENOMEM; }
  if (hipMemset(m->d_w, 0, 2 * kMlpH * kMlpIn * sizeof(unsigned short)) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    gbr_mlp_destroy(m);
    return GBR_EDEVICE;
  }
  *out = m;
  return GBR_OK;
}

int gbr_mlp_destroy(gbr_mlp* m) {
  if (!m) return GBR_OK;
  (void)hipDeviceSynchronize();
  for (void* p : {(void*)m->d_master, (void*)m->d_m, (void*)m->d_v, (void*)m->d_w, (void*)m->d_f,
                  (void*)m->d_partial, (void*)m->d_grad})
    if (p) (void)hipFree(p);
  delete m;
  return GBR_OK;
}

int gbr_mlp_set_params(gbr_mlp* m, const float* w, const float* b) {
  if (!m || !w || !b) return GBR_EINVAL;
  if (hipMemcpy(m->d_master, w, kMlpNW * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(m->d_master + kMlpNW, b, kMlpNB * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(m->d_m, 0, kMlpNP * sizeof(float)) != hipSuccess ||
      hipMemset(m->d_v, 0, kMlpNP * sizeof(float)) != hipSuccess)
    return GBR_EDEVICE;
  m->t = 0;
  hipLaunchKernelGGL(mlp_publish_kernel, dim3((kMlpNP + 255) / 256), dim3(256), 0, 0, m->d_master,
                     m->d_w, m->d_w + kMlpH * kMlpIn, m->d_f, m->d_f + kMlpH);
  return hip_ok(hipDeviceSynchronize());
}

int gbr_mlp_get_params(gbr_mlp* m, float* w, float* b) {
  if (!m) return GBR_EINVAL;
  if (hipDeviceSynchronize() != hipSuccess) return GBR_EDEVICE;
  if (w && hipMemcpy(w, m->d_master, kMlpNW * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
    return GBR_EDEVICE;
  if (b && hipMemcpy(b, m->d_master + kMlpNW, kMlpNB * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
    return GBR_EDEVICE;
  return GBR_OK;
}

static MlpImage mlp_image(const gbr_mlp* m) {
  MlpImage M;
  M.W1 = m->d_w;
  M.W2 = m->d_w + kMlpH * kMlpIn;
  M.w3 = m->d_f;
  M.b = m->d_f + kMlpH;
  return M;
}

int gbr_mlp_features(gbr_ctx* c, const double* Q, uint16_t* feat, uint8_t* chi, void* stream) {
  if (!c || !Q || !feat) return GBR_EINVAL;
  MlpFeatParams P{};
  P.Q = Q; P.feat = feat; P.chi = chi;
  P.nx = c->nx; P.ny = c->ny; P.bcx = c->bcx; P.bcy = c->bcy; P.gamma = c->gamma;
  const size_t n = (size_t)c->nx * c->ny;   // one thread per cell, both directions
  hipLaunchKernelGGL(mlp_features_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, P);
  return hip_ok(hipGetLastError());
}

int gbr_mlp_forward(gbr_mlp* m, const uint16_t* feat, int n, float* logits, void* stream) {
  if (!m || !feat || !logits || n <= 0) return GBR_EINVAL;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                     mlp_image(m), feat, n, logits);
  return hip_ok(hipGetLastError());
}

int gbr_mlp_grad(gbr_mlp* m, const uint16_t* feat, const uint8_t* labels, const int* idx,
                 int batch, float* grad, void* stream) {
  if (!m || !feat || !labels || !idx || !grad) return GBR_EINVAL;
  if (batch <= 0 || batch > kMlpMaxBatch) return GBR_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  MlpGradParams P;
  P.M = mlp_image(m);
  P.feat = feat; P.label = labels; P.idx = idx; P.batch = batch; P.partial = m->d_partial;
  const int nblk = (batch + 255) / 256;
  hipLaunchKernelGGL(mlp_grad_kernel, dim3(nblk), dim3(256), 0, s, P);
  hipLaunchKernelGGL(mlp_sum_kernel, dim3((kMlpNP + 1 + 255) / 256), dim3(256), 0, s,
                     (const float*)m->d_partial, nblk, grad);
  return hip_ok(hipGetLastError());
}

int gbr_mlp_train_step(gbr_mlp* m, const uint16_t* feat, const uint8_t* labels, const int* idx,
                       int batch, float lr, float* loss, void* stream) {
  if (!(lr > 0.f)) return GBR_EINVAL;
  int rc = gbr_mlp_grad(m, feat, labels, idx, batch, m ? m->d_grad : nullptr, stream);
  if (rc != GBR_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  m->t += 1;
  AdamParams A;
  A.grad = m->d_grad; A.master = m->d_master; A.m = m->d_m; A.v = m->d_v;
  A.W1 = m->d_w; A.W2 = m->d_w + kMlpH * kMlpIn; A.w3 = m->d_f; A.b = m->d_f + kMlpH;
  A.lr = lr; A.beta1 = 0.9f; A.beta2 = 0.999f; A.eps = 1e-8f;
  A.bc1 = 1.0f - powf(0.9f, (float)m->t);
  A.bc2 = 1.0f - powf(0.999f, (float)m->t);
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((kMlpNP + 255) / 256), dim3(256), 0, s, A);
  if (loss && hipMemcpyAsync(loss, m->d_grad + kMlpNP, sizeof(float), hipMemcpyDefault, s) != hipSuccess)
    return GBR_EDEVICE;
  return hip_ok(hipGetLastError());
}

int gbr_set_mlp_detector(gbr_ctx* c, const gbr_mlp* m, float margin, void* stream) {
  if (!c || !m || !(margin >= 0.f)) return GBR_EINVAL;
  if (!c->d_mlp_w) {
    if (hipMalloc(&c->d_mlp_w, 2 * kMlpH * kMlpIn * sizeof(unsigned short)) != hipSuccess ||
        hipMalloc(&c->d_mlp_f, (kMlpH + kMlpNB) * sizeof(float)) != hipSuccess ||
        hipMalloc(&c->d_chimap, (size_t)c->nx * c->ny) != hipSuccess ||
        hipMalloc(&c->d_mlp_fb, sizeof(unsigned long long)) != hipSuccess)
      return GBR_ENOMEM;
    if (hipMemset(c->d_mlp_fb, 0, sizeof(unsigned long long)) != hipSuccess) return GBR_EDEVICE;
    c->mlp_evaluated = 0;
  }
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(c->d_mlp_w, m->d_w, 2 * kMlpH * kMlpIn * sizeof(unsigned short),
                     hipMemcpyDeviceToDevice, s) != hipSuccess ||
      hipMemcpyAsync(c->d_mlp_f, m->d_f, (kMlpH + kMlpNB) * sizeof(float), hipMemcpyDeviceToDevice,
                     s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return GBR_EDEVICE;
  c->mlp_margin = margin;
  c->mlp_ready = 1;
  return GBR_OK;
}

int gbr_set_mlp_reuse(gbr_ctx* c, int per_step) {
  if (!c || (per_step != 0 && per_step != 1)) return GBR_EINVAL;
  if (per_step && !c->d_rp &&
      hipMalloc(&c->d_rp, 2 * (size_t)c->nx * c->ny * sizeof(float)) != hipSuccess) {
    c->d_rp = nullptr;
    return GBR_ENOMEM;
  }
  c->mlp_reuse = per_step;
  c->rp_valid = 0;
  c->rp_armed = 0;
  return GBR_OK;
}

int gbr_mlp_get_flagmap(gbr_ctx* c, uint8_t* chi, void* stream) {
  if (!c || !chi || !c->d_chimap) return GBR_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(chi, c->d_chimap, (size_t)c->nx * c->ny, hipMemcpyDefault, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return GBR_EDEVICE;
  return GBR_OK;
}

int gbr_selftest_reciprocal(uint32_t lo, uint32_t hi, uint64_t* mismatches) {
  if (!mismatches || lo > hi) return GBR_EINVAL;
  unsigned long long* d = nullptr;
  if (hipMalloc(&d, sizeof(*d)) != hipSuccess) return GBR_ENOMEM;
  unsigned long long h = 0;
  bool ok = hipMemset(d, 0, sizeof(*d)) == hipSuccess;
  if (ok && hi > lo) {
    hipLaunchKernelGGL(rcp_selftest_kernel, dim3(8192), dim3(256), 0, 0, lo, hi, d);
    ok = hipGetLastError() == hipSuccess;
  }
  ok = ok && hipDeviceSynchronize() == hipSuccess &&
       hipMemcpy(&h, d, sizeof(h), hipMemcpyDeviceToHost) == hipSuccess;
  (void)hipFree(d);
  if (!ok) return GBR_EDEVICE;
  *mismatches = h;
  return GBR_OK;
}

int gbr_selftest_division(uint64_t seed, uint64_t count, uint64_t* mismatches) {
  if (!mismatches) return GBR_EINVAL;
  unsigned long long* d = nullptr;
  if (hipMalloc(&d, sizeof(*d)) != hipSuccess) return GBR_ENOMEM;
  unsigned long long h = 0;
  bool ok = hipMemset(d, 0, sizeof(*d)) == hipSuccess;
  if (ok && count > 0) {
    hipLaunchKernelGGL(div_selftest_kernel, dim3(8192), dim3(256), 0, 0, (unsigned long long)seed,
                       (unsigned long long)count, d);
    ok = hipGetLastError() == hipSuccess;
  }
  ok = ok && hipDeviceSynchronize() == hipSuccess &&
       hipMemcpy(&h, d, sizeof(h), hipMemcpyDeviceToHost) == hipSuccess;
  (void)hipFree(d);
  if (!ok) return GBR_EDEVICE;
  *mismatches = h;
  return GBR_OK;
}

int gbr_mlp_stats(gbr_ctx* c, uint64_t* evaluated, uint64_t* fallbacks, int reset) {
  if (!c || !c->d_mlp_fb) return GBR_EINVAL;
  unsigned long long h = 0;
  if (hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(&h, c->d_mlp_fb, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess)
    return GBR_EDEVICE;
  if (evaluated) *evaluated = c->mlp_evaluated;
  if (fallbacks) *fallbacks = h;
  if (reset) {
    c->mlp_evaluated = 0;
    if (hipMemset(c->d_mlp_fb, 0, sizeof(h)) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
      return GBR_EDEVICE;
  }
  return GBR_OK;
}

// ---------------------------------------------------------------------------
// Batched grids.
struct gbr_batch {
  int nprob, device, precision;
  std::vector<BatchProb> hprob;     // host copy (pointers filled by set_arrays)
  BatchProb* d_prob;
  StageParams* d_tab;               // [9][nprob]: (array roles of the step, stage) -> parameters
  int* d_tile_start;                // [nprob + 1]
  double* d_dt;                     // [nprob]
  double* d_partial;                // [nprob][2][kBatchDtBlocks]
  unsigned* d_status;               // [4]
  int tiling, total, grid, cus;
  int arrays, cur;                  // arrays registered; index of the set holding the state
  int use_graph;
  hipGraphExec_t exec[3];
  hipGraph_t graph[3];
  int timing;                       // gbr_batch_timing: events around stage launches
  std::vector<hipEvent_t> ev;
  size_t ev_used;
};

static void batch_drop_graphs(gbr_batch* b) {
  for (int k = 0; k < 3; ++k) {
    if (b->exec[k]) (void)hipGraphExecDestroy(b->exec[k]);
    if (b->graph[k]) (void)hipGraphDestroy(b->graph[k]);
    b->exec[k] = nullptr;
    b->graph[k] = nullptr;
  }
}

// Tile table and launch size for the current tile shape.
static int batch_layout(gbr_batch* b) {
  const BatchVariant& v = kBatchVariants[b->tiling];
  std::vector<int> ts(b->nprob + 1);
  long long t = 0;
  for (int p = 0; p < b->nprob; ++p) {
    BatchProb& g = b->hprob[p];
    g.tiles_x = (g.nx + v.tx - 1) / v.tx;
    ts[p] = (int)t;
    t += (long long)g.tiles_x * ((g.ny + v.ty - 1) / v.ty);
    if (t > 0x7fffffffll) return GBR_EINVAL;
  }
  ts[b->nprob] = (int)t;
  b->total = (int)t;
  const long long need = (t + 7) / 8 * 8;   // one workgroup per tile (rounded to 8)
  if (v.loop) {
    const int per_cu = v.occ[b->precision == GBR_PREC_FP32_BULK ? 1 : 0]();
    if (per_cu < 1) return GBR_EDEVICE;
    long long g = (long long)per_cu * b->cus;
    g = g / 8 * 8;
    if (g < 8) g = 8;
    b->grid = (int)(g < need ? g : need);
  } else {
    b->grid = (int)need;
  }
  // stage parameter tables: step from set x, stage st (1..3) -> table 3 x + st - 1
  std::vector<StageParams> tab((size_t)9 * b->nprob);
  for (int x = 0; x < 3; ++x) {
    const int y = (x + 1) % 3, z = (x + 2) % 3;
    const int roles[3][2] = {{x, y}, {y, z}, {z, y}};   // (Q^(k), Q^(k+1)) of stages 1..3
    for (int st = 0; st < 3; ++st)
      for (int p = 0; p < b->nprob; ++p) {
        const BatchProb& g = b->hprob[p];
        StageParams& P = tab[(size_t)(3 * x + st) * b->nprob + p];
        P = StageParams{};
        P.Qn = g.buf[x];
        P.Qk = g.buf[roles[st][0]];
        P.out = g.buf[roles[st][1]];
        P.dt = b->d_dt + p;
        P.status = b->d_status;
        P.nx = g.nx; P.ny = g.ny; P.bcx = g.bcx; P.bcy = g.bcy;
        P.tiles_x = g.tiles_x;
        P.ntiles = g.tiles_x * ((g.ny + v.ty - 1) / v.ty);
        P.inv_dx = g.inv_dx; P.inv_dy = g.inv_dy;
        P.gamma = g.gamma; P.g1inv = g.g1inv; P.mu = g.mu; P.kq = g.kq;
        P.mode = MODE_STAGE1 + st;
      }
  }
  if (hipMemcpy(b->d_tile_start, ts.data(), sizeof(int) * (b->nprob + 1), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(b->d_prob, b->hprob.data(), sizeof(BatchProb) * b->nprob,
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->d_tab, tab.data(), sizeof(StageParams) * tab.size(), hipMemcpyHostToDevice) !=
          hipSuccess)
    return GBR_EDEVICE;
  batch_drop_graphs(b);
  return GBR_OK;
}

static void batch_launch_dt(gbr_batch* b, int qn, hipStream_t s) {
  hipLaunchKernelGGL(batch_dt_reduce_kernel, dim3(b->nprob * kBatchDtBlocks), dim3(kDtThreads), 0, s,
                     b->d_prob, qn, b->d_partial, b->d_status);
  hipLaunchKernelGGL(batch_dt_finish_kernel, dim3((b->nprob + 255) / 256), dim3(256), 0, s,
                     b->d_prob, b->nprob, b->d_partial, b->d_dt, b->d_status);
}

// Stage st (1..3) of a step from array set x.
static void batch_launch_stage(gbr_batch* b, int x, int st, hipStream_t s) {
  BatchParams B{};
  B.tab = b->d_tab + (size_t)(3 * x + st - 1) * b->nprob;
  B.tile_start = b->d_tile_start;
  B.nprob = b->nprob;
  B.total = b->total;
  kBatchVariants[b->tiling].fn[b->precision == GBR_PREC_FP32_BULK ? 1 : 0](B, b->grid, s);
}

// One SSP-RK3 step from array set x: stages into y, z, y (y = x+1, z = x+2
// mod 3); the state ends in y.
static int batch_enqueue_step(gbr_batch* b, int x, hipStream_t s) {
  batch_launch_dt(b, x, s);
  for (int st = 1; st <= 3; ++st) {
    hipEvent_t* e = nullptr;
    if (b->timing) {
      if (b->ev_used + 2 > b->ev.size()) {
        for (int k = 0; k < 2 * 64; ++k) {
          hipEvent_t h;
          if (hipEventCreate(&h) != hipSuccess) return GBR_EDEVICE;
          b->ev.push_back(h);
        }
      }
      e = &b->ev[b->ev_used];
      b->ev_used += 2;
      if (hipEventRecord(e[0], s) != hipSuccess) return GBR_EDEVICE;
    }
    batch_launch_stage(b, x, st, s);
    if (e && hipEventRecord(e[1], s) != hipSuccess) return GBR_EDEVICE;
  }
  return GBR_OK;
}

int gbr_batch_init(int nprob, const int* nx, const int* ny, const double* geom, const int* bc,
                   const double* gamma, const double* mu, const double* Pr, const double* cfl,
                   int precision, gbr_batch** out) {
  if (!out || nprob < 1 || !nx || !ny || !geom || !bc || !gamma || !mu || !Pr || !cfl)
    return GBR_EINVAL;
  if (precision != GBR_PREC_FP64 && precision != GBR_PREC_FP32_BULK) return GBR_EINVAL;
  *out = nullptr;
  for (int p = 0; p < nprob; ++p) {
    if (nx[p] < 12 || ny[p] < 12 || !(gamma[p] > 1.0) || !(mu[p] >= 0.0) || !(Pr[p] > 0.0) ||
        !(cfl[p] > 0.0) || !(geom[4 * p + 1] > geom[4 * p]) || !(geom[4 * p + 3] > geom[4 * p + 2]))
      return GBR_EINVAL;
    for (int d = 0; d < 2; ++d)
      if (bc[2 * p + d] != GBR_BC_PERIODIC && bc[2 * p + d] != GBR_BC_TRANSMISSIVE) return GBR_EINVAL;
  }
  gbr_batch* b = new (std::nothrow) gbr_batch();
  if (!b) return GBR_ENOMEM;
  b->nprob = nprob;
  b->precision = precision;
  b->use_graph = 1;
  if (hipGetDevice(&b->device) != hipSuccess ||
      hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, b->device) !=
          hipSuccess) {
    delete b;
    return GBR_EDEVICE;
  }
  b->hprob.resize(nprob);
  for (int p = 0; p < nprob; ++p) {
    BatchProb& g = b->hprob[p];
    g = BatchProb{};
    g.nx = nx[p]; g.ny = ny[p]; g.bcx = bc[2 * p]; g.bcy = bc[2 * p + 1];
    g.dx = (geom[4 * p + 1] - geom[4 * p]) / nx[p];
    g.dy = (geom[4 * p + 3] - geom[4 * p + 2]) / ny[p];
    g.inv_dx = (double)nx[p] / (geom[4 * p + 1] - geom[4 * p]);
    g.inv_dy = (double)ny[p] / (geom[4 * p + 3] - geom[4 * p + 2]);
    g.gamma = gamma[p]; g.g1inv = 1.0 / (gamma[p] - 1.0); g.mu = mu[p];
    g.kq = mu[p] / (Pr[p] * (gamma[p] - 1.0));
    g.cfl = cfl[p];
  }
  if (hipMalloc(&b->d_prob, sizeof(BatchProb) * nprob) != hipSuccess ||
      hipMalloc(&b->d_tab, sizeof(StageParams) * 9 * nprob) != hipSuccess ||
      hipMalloc(&b->d_tile_start, sizeof(int) * (nprob + 1)) != hipSuccess ||
      hipMalloc(&b->d_dt, sizeof(double) * nprob) != hipSuccess ||
      hipMalloc(&b->d_partial, sizeof(double) * 2 * kBatchDtBlocks * nprob) != hipSuccess ||
      hipMalloc(&b->d_status, 4 * sizeof(unsigned)) != hipSuccess ||
      hipMemset(b->d_status, 0, 4 * sizeof(unsigned)) != hipSuccess ||
      hipMemset(b->d_dt, 0, sizeof(double) * nprob) != hipSuccess) {
    gbr_batch_destroy(b);
    return GBR_ENOMEM;
  }
  const int rc = batch_layout(b);
  if (rc != GBR_OK) {
    gbr_batch_destroy(b);
    return rc;
  }
  *out = b;
  return GBR_OK;
}

int gbr_batch_destroy(gbr_batch* b) {
  if (!b) return GBR_OK;
  (void)hipDeviceSynchronize();
  batch_drop_graphs(b);
  for (hipEvent_t e : b->ev) (void)hipEventDestroy(e);
  if (b->d_prob) (void)hipFree(b->d_prob);
  if (b->d_tab) (void)hipFree(b->d_tab);
  if (b->d_tile_start) (void)hipFree(b->d_tile_start);
  if (b->d_dt) (void)hipFree(b->d_dt);
  if (b->d_partial) (void)hipFree(b->d_partial);
  if (b->d_status) (void)hipFree(b->d_status);
  delete b;
  return GBR_OK;
}

int gbr_batch_set_arrays(gbr_batch* b, double* const* X, double* const* Y, double* const* Z) {
  if (!b || !X || !Y || !Z) return GBR_EINVAL;
  for (int p = 0; p < b->nprob; ++p) {
    if (!X[p] || !Y[p] || !Z[p] || X[p] == Y[p] || Y[p] == Z[p] || X[p] == Z[p]) return GBR_EINVAL;
    b->hprob[p].buf[0] = X[p];
    b->hprob[p].buf[1] = Y[p];
    b->hprob[p].buf[2] = Z[p];
  }
  const int rc = batch_layout(b);
  if (rc != GBR_OK) return rc;
  b->arrays = 1;
  b->cur = 0;
  return GBR_OK;
}

int gbr_batch_tiling_count(void) { return kNumBatchVariants; }

int gbr_batch_set_tiling(gbr_batch* b, int variant) {
  if (!b || variant < 0 || variant >= kNumBatchVariants) return GBR_EINVAL;
  b->tiling = variant;
  return batch_layout(b);
}

int gbr_batch_info(gbr_batch* b, int* tiling, int* tile_x, int* tile_y, int* total_tiles,
                   int* workgroups) {
  if (!b) return GBR_EINVAL;
  if (tiling) *tiling = b->tiling;
  if (tile_x) *tile_x = kBatchVariants[b->tiling].tx;
  if (tile_y) *tile_y = kBatchVariants[b->tiling].ty;
  if (total_tiles) *total_tiles = b->total;
  if (workgroups) *workgroups = b->grid;
  return GBR_OK;
}

int gbr_batch_use_graph(gbr_batch* b, int enable) {
  if (!b) return GBR_EINVAL;
  b->use_graph = enable ? 1 : 0;
  return GBR_OK;
}

int gbr_batch_step(gbr_batch* b, void* stream) {
  if (!b || !b->arrays) return GBR_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const int x = b->cur;
  if (b->use_graph && s && !b->timing) {
    if (!b->exec[x]) {
      if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return GBR_EDEVICE;
      const int rc = batch_enqueue_step(b, x, s);
      if (hipStreamEndCapture(s, &b->graph[x]) != hipSuccess || rc != GBR_OK) return GBR_EDEVICE;
      if (hipGraphInstantiate(&b->exec[x], b->graph[x], nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(b->graph[x]);
        b->graph[x] = nullptr;
        b->exec[x] = nullptr;
        return GBR_EDEVICE;
      }
    }
    if (hipGraphLaunch(b->exec[x], s) != hipSuccess) return GBR_EDEVICE;
  } else {
    const int rc = batch_enqueue_step(b, x, s);
    if (rc != GBR_OK) return rc;
    if (hipGetLastError() != hipSuccess) return GBR_EDEVICE;
  }
  b->cur = (x + 1) % 3;
  return GBR_OK;
}

int gbr_batch_timing(gbr_batch* b, int enable) {
  if (!b) return GBR_EINVAL;
  b->timing = enable ? 1 : 0;
  b->ev_used = 0;
  return GBR_OK;
}

int gbr_batch_timing_read(gbr_batch* b, double* stage_ms, uint64_t* launches) {
  if (!b) return GBR_EINVAL;
  double t = 0.0;
  for (size_t k = 0; k + 2 <= b->ev_used; k += 2) {
    float ms = 0.f;
    if (hipEventSynchronize(b->ev[k + 1]) != hipSuccess ||
        hipEventElapsedTime(&ms, b->ev[k], b->ev[k + 1]) != hipSuccess)
      return GBR_EDEVICE;
    t += ms;
  }
  if (stage_ms) *stage_ms = t;
  if (launches) *launches = b->ev_used / 2;
  b->ev_used = 0;
  return GBR_OK;
}

int gbr_batch_current(gbr_batch* b, int* which) {
  if (!b || !which) return GBR_EINVAL;
  *which = b->cur;
  return GBR_OK;
}

int gbr_batch_get_dt(gbr_batch* b, double* dt, void* stream) {
  if (!b || !dt) return GBR_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(dt, b->d_dt, sizeof(double) * b->nprob, hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return GBR_EDEVICE;
  return GBR_OK;
}

int gbr_batch_check(gbr_batch* b, void* stream) {
  if (!b) return GBR_EINVAL;
  unsigned h[4] = {0, 0, 0, 0};
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess ||
      hipMemcpy(h, b->d_status, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemset(b->d_status, 0, sizeof(h)) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
    return GBR_EDEVICE;
  return (h[0] | h[1] | h[2] | h[3]) ? GBR_ESTATE : GBR_OK;
}

int gbr_batch_autotune(gbr_batch* b, int reps, void* stream) {
  if (!b || !b->arrays || reps < 1) return GBR_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return GBR_EDEVICE;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return GBR_EDEVICE;
  }
  const int saved = b->tiling, x = b->cur;
  int best = saved, rc = GBR_OK;
  float best_ms = 1e30f;
  for (int v = 0; v < kNumBatchVariants && rc == GBR_OK; ++v) {
    b->tiling = v;
    if ((rc = batch_layout(b)) != GBR_OK) break;
    // first stage of a step from the current state into a scratch set
    batch_launch_dt(b, x, s);
    batch_launch_stage(b, x, 1, s);
    (void)hipEventRecord(e0, s);   // (stage launches here record no timing events)
    for (int r = 0; r < reps; ++r) batch_launch_stage(b, x, 1, s);
    (void)hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess) { rc = GBR_EDEVICE; break; }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms < best_ms) { best_ms = ms; best = v; }
  }
  b->tiling = best;
  const int rc2 = batch_layout(b);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc != GBR_OK ? rc : rc2;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Three dimensions (inviscid): one line-sweep kernel per direction and stage.
namespace {
constexpr int k3NP = 32, k3NL = 8;   // positions per tile along the line, lines per workgroup
using Sweep3Fn = void (*)(const Sweep3Params&, int, hipStream_t);
template <int DIR, int ORD>
void launch_sweep3(const Sweep3Params& P, int grid, hipStream_t s) {
  hipLaunchKernelGGL((meg7_sweep3_kernel<DIR, k3NP, k3NL, ORD>), dim3(grid), dim3(256), 0, s, P);
}
const Sweep3Fn kSweep3[2][3] = {
    {launch_sweep3<0, 7>, launch_sweep3<1, 7>, launch_sweep3<2, 7>},
    {launch_sweep3<0, 4>, launch_sweep3<1, 4>, launch_sweep3<2, 4>}};
// fused x/y forms: 15x15 tiles of a z plane, all 15 lines of a sweep at once
// (two workgroups per CU) or 8 at a time (three)
using XY3Fn = void (*)(const XY3Params&, int, hipStream_t);
template <int NL, int ORD>
void launch_xy3(const XY3Params& P, int grid, hipStream_t s) {
  using C = XY3Cfg<15, 15, NL>;
  static_assert(C::LDS_BYTES <= 160 * 1024, "LDS per workgroup");
  hipLaunchKernelGGL((meg7_xy3_kernel<C, ORD>), dim3(grid), dim3(C::NT), 0, s, P);
}
const XY3Fn kXY3[2][2] = {{launch_xy3<15, 7>, launch_xy3<8, 7>},
                          {launch_xy3<15, 4>, launch_xy3<8, 4>}};
constexpr int kXY3T = 15;   // tile side of the fused forms
}  // namespace

struct gbr3_ctx {
  int n[3];
  double gamma;
  double lo[3], hi[3];
  int bc[3];
  int order;
  int sweeps;                 // GBR3_SWEEPS_*
  int device;
  int export_flags;
  unsigned* d_status;         // [4]
  double* d_partial;          // [2][kDtBlocks]
  double* d_R;                // [5][nz][ny][nx] residual accumulator
  double* d_dtx;              // [3][slots] per-wave time-step extrema of a stage-3 output
  int stage3_slots;           // slots of the last stage-3 call; 0: none since gbr3_stage_dt
  uint8_t* d_sig[3];          // optional interface flags per direction
  int timing;
  std::vector<hipEvent_t> ev; // two per residual or stage call
  size_t ev_used;
};

int gbr3_init(int nx, int ny, int nz, double gamma, gbr3_ctx** out) {
  if (!out) return GBR_EINVAL;
  *out = nullptr;
  if (nx < 12 || ny < 12 || nz < 12 || !(gamma > 1.0)) return GBR_EINVAL;
  if ((long long)nx * ny * nz > (1ll << 31) / 5) return GBR_EINVAL;
  gbr3_ctx* c = new (std::nothrow) gbr3_ctx();
  if (!c) return GBR_ENOMEM;
  c->n[0] = nx; c->n[1] = ny; c->n[2] = nz; c->gamma = gamma;
  for (int d = 0; d < 3; ++d) { c->lo[d] = 0.0; c->hi[d] = 1.0; c->bc[d] = GBR_BC_PERIODIC; }
  c->order = 7;
  c->sweeps = GBR3_SWEEPS_LINES;
  const size_t n = (size_t)nx * ny * nz;
  // the z sweep's workgroups: line groups of the xy plane x position tiles
  const size_t zslots = 4 * (((size_t)nx * ny + k3NL - 1) / k3NL) * ((nz + k3NP - 1) / k3NP);
  bool ok = hipGetDevice(&c->device) == hipSuccess &&
            hipMalloc(&c->d_status, 4 * sizeof(unsigned)) == hipSuccess &&
            hipMalloc(&c->d_partial, 3 * kDtBlocks * sizeof(double)) == hipSuccess &&
            hipMalloc(&c->d_R, 5 * n * sizeof(double)) == hipSuccess &&
            hipMalloc(&c->d_dtx, 3 * zslots * sizeof(double)) == hipSuccess &&
            hipMemset(c->d_status, 0, 4 * sizeof(unsigned)) == hipSuccess &&
            hipDeviceSynchronize() == hipSuccess;
  if (!ok) {
    (void)hipFree(c->d_status); (void)hipFree(c->d_partial); (void)hipFree(c->d_R);
    (void)hipFree(c->d_dtx);
    delete c;
    return GBR_ENOMEM;
  }
  *out = c;
  return GBR_OK;
}

int gbr3_destroy(gbr3_ctx* c) {
  if (!c) return GBR_OK;
  (void)hipDeviceSynchronize();
  (void)hipFree(c->d_status);
  (void)hipFree(c->d_partial);
  (void)hipFree(c->d_R);
  (void)hipFree(c->d_dtx);
  for (int d = 0; d < 3; ++d)
    if (c->d_sig[d]) (void)hipFree(c->d_sig[d]);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  delete c;
  return GBR_OK;
}

int gbr3_set_geometry(gbr3_ctx* c, double x0, double x1, double y0, double y1, double z0,
                      double z1, int bc_x, int bc_y, int bc_z) {
  if (!c || !(x1 > x0) || !(y1 > y0) || !(z1 > z0)) return GBR_EINVAL;
  const int bc[3] = {bc_x, bc_y, bc_z};
  for (int d = 0; d < 3; ++d)
    if (bc[d] != GBR_BC_PERIODIC && bc[d] != GBR_BC_TRANSMISSIVE) return GBR_EINVAL;
  c->lo[0] = x0; c->hi[0] = x1; c->lo[1] = y0; c->hi[1] = y1; c->lo[2] = z0; c->hi[2] = z1;
  for (int d = 0; d < 3; ++d) c->bc[d] = bc[d];
  return GBR_OK;
}

int gbr3_set_order(gbr3_ctx* c, int order) {
  if (!c || (order != 7 && order != 4)) return GBR_EINVAL;
  c->order = order;
  return GBR_OK;
}

int gbr3_set_sweeps(gbr3_ctx* c, int form) {
  if (!c || form < GBR3_SWEEPS_LINES || form > GBR3_SWEEPS_XY_FUSED_HALF) return GBR_EINVAL;
  c->sweeps = form;
  return GBR_OK;
}

int gbr3_export_flags(gbr3_ctx* c, int enable) {
  if (!c) return GBR_EINVAL;
  if (enable) {
    for (int d = 0; d < 3; ++d) {
      if (c->d_sig[d]) continue;
      size_t m = 1;
      for (int e = 0; e < 3; ++e) m *= (size_t)c->n[e] + (e == d ? 1 : 0);
      if (hipMalloc(&c->d_sig[d], m) != hipSuccess) return GBR_ENOMEM;
    }
  }
  c->export_flags = enable ? 1 : 0;
  return GBR_OK;
}

int gbr3_get_flags(gbr3_ctx* c, uint8_t* sig_x, uint8_t* sig_y, uint8_t* sig_z, void* stream) {
  if (!c || !c->d_sig[0]) return GBR_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  uint8_t* dst[3] = {sig_x, sig_y, sig_z};
  for (int d = 0; d < 3; ++d) {
    if (!dst[d]) continue;
    size_t m = 1;
    for (int e = 0; e < 3; ++e) m *= (size_t)c->n[e] + (e == d ? 1 : 0);
    if (hipMemcpyAsync(dst[d], c->d_sig[d], m, hipMemcpyDefault, s) != hipSuccess)
      return GBR_EDEVICE;
  }
  return hip_ok(hipStreamSynchronize(s));
}

int gbr3_check(gbr3_ctx* c, void* stream) {
  if (!c) return GBR_EINVAL;
  unsigned h[4] = {0, 0, 0, 0};
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return GBR_EDEVICE;
  if (hipMemcpy(h, c->d_status, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess)
    return GBR_EDEVICE;
  if (hipMemset(c->d_status, 0, sizeof(h)) != hipSuccess) return GBR_EDEVICE;
  if (hipDeviceSynchronize() != hipSuccess) return GBR_EDEVICE;
  return (h[0] | h[1] | h[2] | h[3]) ? GBR_ESTATE : GBR_OK;
}

static int launch3(gbr3_ctx* c, int mode, const double* dt, const double* Qn, const double* Qk,
                   double* out, hipStream_t s) {
  hipEvent_t* tev = nullptr;
  if (c->timing) {
    if (c->ev_used + 2 > c->ev.size()) {
      for (int k = 0; k < 2 * 64; ++k) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return GBR_EDEVICE;
        c->ev.push_back(e);
      }
    }
    tev = &c->ev[c->ev_used];
    c->ev_used += 2;
    if (hipEventRecord(tev[0], s) != hipSuccess) return GBR_EDEVICE;
  }
  const int o4 = c->order == 4 ? 1 : 0;
  const bool fused = c->sweeps != GBR3_SWEEPS_LINES;
  if (fused) {
    XY3Params X{};
    X.Qk = Qk; X.R = c->d_R;
    X.sigx = c->export_flags ? c->d_sig[0] : nullptr;
    X.sigy = c->export_flags ? c->d_sig[1] : nullptr;
    X.status = c->d_status;
    X.nx = c->n[0]; X.ny = c->n[1]; X.nz = c->n[2]; X.bcx = c->bc[0]; X.bcy = c->bc[1];
    X.tiles_x = (c->n[0] + kXY3T - 1) / kXY3T;
    X.tiles_y = (c->n[1] + kXY3T - 1) / kXY3T;
    const long long nt = (long long)X.tiles_x * X.tiles_y * c->n[2];
    if (nt > 0x7fffffff) return GBR_EINVAL;
    X.ntiles = (int)nt;
    X.inv_dx = (double)c->n[0] / (c->hi[0] - c->lo[0]);
    X.inv_dy = (double)c->n[1] / (c->hi[1] - c->lo[1]);
    X.gamma = c->gamma; X.g1inv = 1.0 / (c->gamma - 1.0);
    kXY3[o4][c->sweeps == GBR3_SWEEPS_XY_FUSED ? 0 : 1](X, X.ntiles, s);
  }
  for (int d = fused ? 2 : 0; d < 3; ++d) {
    Sweep3Params P{};
    P.Qk = Qk; P.Qn = Qn; P.R = c->d_R; P.out = out; P.dt = dt;
    P.sig = c->export_flags ? c->d_sig[d] : nullptr;
    P.status = c->d_status;
    P.nx = c->n[0]; P.ny = c->n[1]; P.nz = c->n[2];
    P.bc = c->bc[d];
    P.inv_d = (double)c->n[d] / (c->hi[d] - c->lo[d]);
    P.gamma = c->gamma; P.g1inv = 1.0 / (c->gamma - 1.0);
    P.first = !fused && d == 0; P.last = d == 2;
    P.mode = mode;
    P.ptiles = (c->n[d] + k3NP - 1) / k3NP;
    const long long lines = (long long)c->n[(d + 1) % 3] * c->n[(d + 2) % 3];
    const long long groups = (lines + k3NL - 1) / k3NL;
    const long long grid = groups * P.ptiles;
    if (grid > 0x7fffffff) return GBR_EINVAL;
    P.dtx = (d == 2 && mode == MODE_STAGE3) ? c->d_dtx : nullptr;
    kSweep3[o4][d](P, (int)grid, s);
    if (P.dtx) c->stage3_slots = (int)grid * 4;
  }
  if (tev && hipEventRecord(tev[1], s) != hipSuccess) return GBR_EDEVICE;
  return hip_ok(hipGetLastError());
}

int gbr3_residual(gbr3_ctx* c, const double* Q, double* Res, void* stream) {
  if (!c || !Q || !Res || Q == Res) return GBR_EINVAL;
  return launch3(c, MODE_RESIDUAL, nullptr, Q, Q, Res, (hipStream_t)stream);
}

int gbr3_rk_stage(gbr3_ctx* c, int stage, const double* dt_dev, const double* Qn,
                  const double* Qk, double* Qout, void* stream) {
  if (!c || !dt_dev || !Qn || !Qk || !Qout) return GBR_EINVAL;
  if (stage < 1 || stage > 3) return GBR_EINVAL;
  if (Qout == Qn || Qout == Qk) return GBR_EINVAL;
  if (stage == 1 && Qk != Qn) return GBR_EINVAL;
  return launch3(c, stage, dt_dev, Qn, Qk, Qout, (hipStream_t)stream);
}

int gbr3_compute_dt(gbr3_ctx* c, const double* Q, double cfl, double* dt_dev, void* stream) {
  if (!c || !Q || !dt_dev || !(cfl > 0.0)) return GBR_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  Dt3Params P{};
  P.Q = Q; P.partial = c->d_partial; P.status = c->d_status;
  P.nx = c->n[0]; P.ny = c->n[1]; P.nz = c->n[2];
  P.dx = (c->hi[0] - c->lo[0]) / c->n[0];
  P.dy = (c->hi[1] - c->lo[1]) / c->n[1];
  P.dz = (c->hi[2] - c->lo[2]) / c->n[2];
  P.gamma = c->gamma;
  const int blocks = dt_blocks((size_t)c->n[0] * c->n[1] * c->n[2]);
  hipLaunchKernelGGL(dt3_reduce_kernel, dim3(blocks), dim3(kDtThreads), 0, s, P);
  hipLaunchKernelGGL(dt_finish_kernel, dim3(1), dim3(kDtThreads), 0, s, c->d_partial, blocks,
                     dt_dev, cfl, c->d_status);
  return hip_ok(hipGetLastError());
}

int gbr3_stage_dt(gbr3_ctx* c, double cfl, double* dt_dev, void* stream) {
  if (!c || !dt_dev || !(cfl > 0.0) || c->stage3_slots <= 0) return GBR_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const int nslot = c->stage3_slots;
  const int blocks = dt_blocks((size_t)nslot);
  hipLaunchKernelGGL(dt_extrema_reduce_kernel<true>, dim3(blocks), dim3(kDtThreads), 0, s,
                     (const double*)c->d_dtx, nslot, c->d_partial);
  hipLaunchKernelGGL(dt3_from_extrema_kernel, dim3(1), dim3(kDtThreads), 0, s,
                     (const double*)c->d_partial, blocks, dt_dev, cfl,
                     (c->hi[0] - c->lo[0]) / c->n[0], (c->hi[1] - c->lo[1]) / c->n[1],
                     (c->hi[2] - c->lo[2]) / c->n[2], c->d_status);
  c->stage3_slots = 0;
  return hip_ok(hipGetLastError());
}

int gbr3_timing(gbr3_ctx* c, int enable) {
  if (!c) return GBR_EINVAL;
  c->timing = enable ? 1 : 0;
  c->ev_used = 0;
  return GBR_OK;
}

int gbr3_timing_read(gbr3_ctx* c, double* sweeps_ms, uint64_t* calls) {
  if (!c) return GBR_EINVAL;
  double t = 0.0;
  for (size_t k = 0; k + 2 <= c->ev_used; k += 2) {
    float a = 0.f;
    if (hipEventSynchronize(c->ev[k + 1]) != hipSuccess ||
        hipEventElapsedTime(&a, c->ev[k], c->ev[k + 1]) != hipSuccess)
      return GBR_EDEVICE;
    t += a;
  }
  if (sweeps_ms) *sweeps_ms = t;
  if (calls) *calls = c->ev_used / 2;
  c->ev_used = 0;
  return GBR_OK;
}
