/* A plain C program that drives the library through include/gbr.h only:
 * device memory from the HIP runtime API, no Python, no torch.
 *
 *   gbr_c_driver IN OUT
 *
 * IN (binary, native endian): int32 nx, ny, bc_x, bc_y; float64 x0, x1, y0,
 * y1, gamma, mu, Pr, cfl; then Q as float64 [4][ny][nx].
 * OUT: int32 status codes of the eight library calls below; float64 dt; then
 * the residual of Q [4][ny][nx], the interface flags of that residual
 * (uint8 [ny][nx+1] then [ny+1][nx]) and the state after one SSP-RK3 step
 * [4][ny][nx] (dt from gbr_compute_dt, stages 1-3 with gbr_rk_stage).
 * Exit status 0 when every call returned GBR_OK, 1 when one did not,
 * 2 for a usage or I/O error (before any HIP call). */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "gbr.h"

static int rd(FILE* f, void* p, size_t sz, size_t n) { return fread(p, sz, n, f) == n; }

int main(int argc, char** argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: %s IN OUT\n", argv[0]);
    return 2;
  }
  FILE* in = fopen(argv[1], "rb");
  if (!in) {
    fprintf(stderr, "cannot open %s\n", argv[1]);
    return 2;
  }
  int32_t hdr[4];
  double par[8];
  if (!rd(in, hdr, sizeof(int32_t), 4) || !rd(in, par, sizeof(double), 8)) {
    fprintf(stderr, "short header\n");
    fclose(in);
    return 2;
  }
  const int nx = hdr[0], ny = hdr[1];
  if (nx < 1 || ny < 1 || (long long)nx * ny > (1ll << 26)) {
    fprintf(stderr, "bad grid %d x %d\n", nx, ny);
    fclose(in);
    return 2;
  }
  const size_t n = (size_t)nx * ny, bytes = 4 * n * sizeof(double);
  double* hQ = (double*)malloc(bytes);
  double* hR = (double*)malloc(bytes);
  double* hQ1 = (double*)malloc(bytes);
  uint8_t* sx = (uint8_t*)malloc((size_t)ny * (nx + 1));
  uint8_t* sy = (uint8_t*)malloc((size_t)(ny + 1) * nx);
  if (!hQ || !hR || !hQ1 || !sx || !sy || !rd(in, hQ, sizeof(double), 4 * n)) {
    fprintf(stderr, "short state or no memory\n");
    fclose(in);
    return 2;
  }
  fclose(in);

  int32_t st[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  double *dQ = NULL, *dR = NULL, *dQ1 = NULL, *dQ2 = NULL, *dQ3 = NULL, *ddt = NULL;
  if (hipMalloc((void**)&dQ, bytes) != hipSuccess || hipMalloc((void**)&dR, bytes) != hipSuccess ||
      hipMalloc((void**)&dQ1, bytes) != hipSuccess || hipMalloc((void**)&dQ2, bytes) != hipSuccess ||
      hipMalloc((void**)&dQ3, bytes) != hipSuccess ||
      hipMalloc((void**)&ddt, sizeof(double)) != hipSuccess ||
      hipMemcpy(dQ, hQ, bytes, hipMemcpyHostToDevice) != hipSuccess) {
    fprintf(stderr, "device allocation or copy failed\n");
    return 1;
  }
  gbr_ctx* ctx = NULL;
  st[0] = gbr_init(nx, ny, par[4], par[5], par[6], &ctx);
  if (st[0] == GBR_OK) {
    st[1] = gbr_set_geometry(ctx, par[0], par[1], par[2], par[3], hdr[2], hdr[3]);
    st[2] = gbr_export_flags(ctx, 1);
    st[3] = gbr_residual(ctx, dQ, dR, NULL);
    st[4] = gbr_get_flags(ctx, sx, sy, NULL);
    st[5] = gbr_compute_dt(ctx, dQ, par[7], ddt, NULL);
    int s6 = gbr_rk_stage(ctx, 1, ddt, dQ, dQ, dQ1, NULL);
    if (s6 == GBR_OK) s6 = gbr_rk_stage(ctx, 2, ddt, dQ, dQ1, dQ2, NULL);
    if (s6 == GBR_OK) s6 = gbr_rk_stage(ctx, 3, ddt, dQ, dQ2, dQ3, NULL);
    st[6] = s6;
    st[7] = gbr_check(ctx, NULL);
  }
  double dt = 0.0;
  int ok = hipDeviceSynchronize() == hipSuccess &&
           hipMemcpy(hR, dR, bytes, hipMemcpyDeviceToHost) == hipSuccess &&
           hipMemcpy(hQ1, dQ3, bytes, hipMemcpyDeviceToHost) == hipSuccess &&
           hipMemcpy(&dt, ddt, sizeof(double), hipMemcpyDeviceToHost) == hipSuccess;
  if (ctx) gbr_destroy(ctx);
  hipFree(dQ); hipFree(dR); hipFree(dQ1); hipFree(dQ2); hipFree(dQ3); hipFree(ddt);
  if (!ok) {
    fprintf(stderr, "device copy failed\n");
    return 1;
  }
  FILE* out = fopen(argv[2], "wb");
  if (!out) {
    fprintf(stderr, "cannot open %s\n", argv[2]);
    return 2;
  }
  fwrite(st, sizeof(int32_t), 8, out);
  fwrite(&dt, sizeof(double), 1, out);
  fwrite(hR, sizeof(double), 4 * n, out);
  fwrite(sx, 1, (size_t)ny * (nx + 1), out);
  fwrite(sy, 1, (size_t)(ny + 1) * nx, out);
  fwrite(hQ1, sizeof(double), 4 * n, out);
  fclose(out);
  free(hQ); free(hR); free(hQ1); free(sx); free(sy);
  for (int k = 0; k < 8; ++k)
    if (st[k] != GBR_OK) {
      fprintf(stderr, "call %d: %s\n", k, gbr_strerror(st[k]));
      return 1;
    }
  return 0;
}
