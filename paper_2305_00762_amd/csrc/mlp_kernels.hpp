// Learned discontinuity detector: per-cell features, an MLP 28 -> 32 -> 32 -> 1
// (bf16 weights, fp32 accumulation on the matrix cores), its training
// (forward, backward, Adam) and its inference.
//
// Matrix-core layout.  v_mfma_f32_16x16x16_bf16 multiplies a 16x16 A (M x K)
// by a 16x16 B (K x N).  In a wave, lane l = 16 g + r (g = 0..3, r = 0..15)
// supplies A[r][4g..4g+3] and B[4g..4g+3][r] and receives D[4g..4g+3][r].
// The network is evaluated transposed, hidden = W x^T: A is a weight block
// (rows = neurons), B an activation block (columns = 16 cells).  The output of
// one layer (lane holds neurons 4g..4g+3 of cell r) is then exactly the B
// operand of the next layer, so activations never leave registers.
#pragma once
#include "meg7_device.hpp"

namespace gbr {

constexpr int kMlpF = 28;             // features
constexpr int kMlpIn = 32;            // padded input width
constexpr int kMlpH = 32;             // hidden width
constexpr int kMlpNW = kMlpH * kMlpF + kMlpH * kMlpH + kMlpH;   // 1952 weights
constexpr int kMlpNB = 2 * kMlpH + 1;                            // 65 biases
constexpr int kMlpNP = kMlpNW + kMlpNB;                          // 2017 parameters
constexpr int kMlpWB = 2 * kMlpH * kMlpIn + kMlpH;               // bf16 inference image

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4f mfma16(v4s a, v4s b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// float32 -> bfloat16, round to nearest even (finite inputs)
__device__ __forceinline__ unsigned short f2bf(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float((unsigned)b << 16); }

__device__ __forceinline__ v4s pack4(float a, float b, float c, float d) {
  v4s r;
  r[0] = (short)f2bf(a); r[1] = (short)f2bf(b); r[2] = (short)f2bf(c); r[3] = (short)f2bf(d);
  return r;
}

// float32 pair -> packed bf16 pair (low half = a), round to nearest even, by
// the hardware conversion (same result as f2bf for finite values).
__device__ __forceinline__ unsigned cvt_pk_bf16(float a, float b) {
  typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
  bf2 r;
  r[0] = (__bf16)a;
  r[1] = (__bf16)b;
  return __builtin_bit_cast(unsigned, r);
}

// 1/x rounded to nearest for normal x with a normal reciprocal (x in
// [2^-126, 2^126)): the hardware estimate and one Newton step with fused
// multiply-adds.  An exhaustive run over all such floats (2^31 - 2^24 of
// them) on gfx950 matches IEEE division bit for bit (gbr_selftest_reciprocal
// repeats it).
__device__ __forceinline__ float rcp_rn(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return __builtin_fmaf(__builtin_fmaf(-x, r, 1.0f), r, r);
}

// Features of one cell.  val(s, o) returns the stencil value at offset o
// (-3..3) of stencil s: 0 rho along x, 1 p along x, 2 rho along y, 3 p along
// y.  Each stencil is taken to float32 and normalised as
// (s_k - mean) / ((max - min) + 1e-3) with a fixed operation order (sum left
// to right, mean = sum * fl(1/7), one correctly rounded reciprocal), then rounded to bf16.
// out[j] holds features 2j (low half) and 2j+1; out[14], out[15] are zero.
template <class FV>
__device__ __forceinline__ void mlp_cell_features(FV val, unsigned out[kMlpIn / 2]) {
#pragma clang fp contract(off)
  float f[kMlpF];
  int col = 0;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    float v[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) v[k] = (float)val(s, k - 3);
    float tot = v[0];
#pragma unroll
    for (int k = 1; k < 7; ++k) tot = tot + v[k];
    const float mean = tot * (1.0f / 7.0f);
    float mx = v[0], mn = v[0];
#pragma unroll
    for (int k = 1; k < 7; ++k) { mx = fmaxf(mx, v[k]); mn = fminf(mn, v[k]); }
    const float d = (mx - mn) + 1e-3f;
    const float r = d < 0x1p126f ? rcp_rn(d) : 1.0f / d;
#pragma unroll
    for (int k = 0; k < 7; ++k) f[col++] = (v[k] - mean) * r;
  }
#pragma unroll
  for (int j = 0; j < kMlpF / 2; ++j) out[j] = cvt_pk_bf16(f[2 * j], f[2 * j + 1]);
  out[kMlpF / 2] = 0;
  out[kMlpF / 2 + 1] = 0;
}

// Inference image of the network: bf16 W1 [32][32] (inputs 28..31 zero), bf16
// W2 [32][32], then float32 w3 [32] (bf16-valued), b1 [32], b2 [32], b3.
struct MlpImage {
  const unsigned short* W1;
  const unsigned short* W2;
  const float* w3;
  const float* b;   // [65]
};

// Per-lane weight fragments and bias/output weights in the D layout.
struct MlpFrags {
  v4s a1[2][2], a2[2][2];   // [neuron block][k step]
  float b1[2][4], b2[2][4], w3[2][4];
  float b3;
};

__device__ __forceinline__ void mlp_load_frags(const MlpImage& M, MlpFrags& F) {
  const int l = __lane_id(), r = l & 15, g = l >> 4;
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const int n = 16 * nb + r, k = 16 * ks + 4 * g;
      F.a1[nb][ks] = *reinterpret_cast<const v4s*>(M.W1 + n * kMlpIn + k);
      F.a2[nb][ks] = *reinterpret_cast<const v4s*>(M.W2 + n * kMlpH + k);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int n = 16 * nb + 4 * g + i;
      F.b1[nb][i] = M.b[n];
      F.b2[nb][i] = M.b[kMlpH + n];
      F.w3[nb][i] = M.w3[n];
    }
  }
  F.b3 = M.b[2 * kMlpH];
}

// Inference on the K = 32 matrix instruction (v_mfma_f32_16x16x32_bf16):
// lane l = 16 g + r supplies 8 bf16 of row r of A and of column r of B, for
// one group of 8 K indices per g, and receives D[4g..4g+3][r] as before.
// Which K indices a (g, element) slot stands for does not matter as long as A
// and B fill the slot with the same index: the slot of lane group g, element
// e holds feature 8g + e in layer 1 and hidden neuron 16 (e / 4) + 4 g + e % 4
// in layer 2 -- exactly the layer-1 output the lane already holds, so the
// hidden activations go from the accumulator to the next B operand in
// registers.  The biases initialise the accumulators.
typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

__device__ __forceinline__ v4f mfma32(v8s a, v8s b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a),
                                                 __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
}

// ReLU of two packed bf16 values: a negative bf16 is a negative 16-bit
// integer, so a packed integer max with zero clears it.  bf16(relu(x)) equals
// relu(bf16(x)) for every x (rounding keeps the sign), so converting first
// and clearing after gives the same bits as the other order.
__device__ __forceinline__ unsigned relu_bf16x2(unsigned v) {
  // an empty asm keeps the packed conversion that produced v whole: without
  // it the compiler splits the conversion into two single ones and a permute
  asm("" : "+v"(v));
  typedef short s2 __attribute__((ext_vector_type(2)));
  const s2 x = __builtin_elementwise_max(__builtin_bit_cast(s2, v), (s2){0, 0});
  return __builtin_bit_cast(unsigned, x);
}

// The evaluation along y feeds the same staged (x-order) features: its input
// is the x-order vector with the two stencil halves (features 0..13 and
// 14..27) swapped, so W1 with its columns swapped the same way (a1y) gives
// the y-evaluation's first layer.
//
// The output layer runs on the matrix cores too: its A operand holds w3 (in
// the slot order of the hidden layer) in every row, so every row of the
// product holds the logits of the 16 cells, and lane l = 16 g + r receives
// the logit of cell r in all four accumulator elements.  Its B operand is
// relu(h2) rounded to bf16, packed like the layer-1 output.
struct MlpInfer {
  v8s a1[2], a1y[2], a2[2];   // [neuron block]
  v8s a3;                     // w3 in slot order (the same in every row)
  v4f b1[2], b2[2];   // biases of neurons 16 nb + 4 g + i
  float b3;
};

__device__ __forceinline__ void mlp_load_infer(const MlpImage& M, MlpInfer& F) {
  const int l = __lane_id(), r = l & 15, g = l >> 4;
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    const int n = 16 * nb + r;
    F.a1[nb] = *reinterpret_cast<const v8s*>(M.W1 + n * kMlpIn + 8 * g);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = 8 * g + e;
      F.a1y[nb][e] = (short)M.W1[n * kMlpIn + (k < kMlpF ? (k + kMlpF / 2) % kMlpF : k)];
    }
    const v4s lo = *reinterpret_cast<const v4s*>(M.W2 + n * kMlpH + 4 * g);
    const v4s hi = *reinterpret_cast<const v4s*>(M.W2 + n * kMlpH + 16 + 4 * g);
    F.a2[nb] = (v8s){lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = 16 * nb + 4 * g + i;
      F.b1[nb][i] = M.b[m];
      F.b2[nb][i] = M.b[kMlpH + m];
      F.a3[4 * nb + i] = (short)f2bf(M.w3[m]);   // w3 is bf16-valued: exact
    }
  }
  F.b3 = M.b[2 * kMlpH];
}

// Logit of the 16 cells whose features (slot layout above) lanes hold in x;
// cell r = lane & 15 (the same value in the four lanes of a column).  ydir:
// evaluate along y from the x-order features.
__device__ __forceinline__ float mlp_infer16(const MlpInfer& F, v8s x, bool ydir = false) {
  unsigned hp[4];
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    const v4f c = mfma32(ydir ? F.a1y[nb] : F.a1[nb], x, F.b1[nb]);
    hp[2 * nb] = relu_bf16x2(cvt_pk_bf16(c[0], c[1]));
    hp[2 * nb + 1] = relu_bf16x2(cvt_pk_bf16(c[2], c[3]));
  }
  const v8s h = __builtin_bit_cast(v8s, (uint4){hp[0], hp[1], hp[2], hp[3]});
  unsigned qp[4];
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    const v4f c = mfma32(F.a2[nb], h, F.b2[nb]);
    qp[2 * nb] = relu_bf16x2(cvt_pk_bf16(c[0], c[1]));
    qp[2 * nb + 1] = relu_bf16x2(cvt_pk_bf16(c[2], c[3]));
  }
  const v8s h2 = __builtin_bit_cast(v8s, (uint4){qp[0], qp[1], qp[2], qp[3]});
  const v4f z = mfma32(F.a3, h2, (v4f){F.b3, F.b3, F.b3, F.b3});
  return z[0];
}

// Forward pass of 16 cells whose bf16 B fragments (k steps 0, 1) are x0, x1.
// Returns the logit of cell r = lane & 15 (the same in the four lanes of a
// column); a1/a2 (pre-activations) and h (bf16 h1 fragments) on request.
struct MlpFwdState {
  v4f a1[2], a2[2];
  v4s h[2];
};
__device__ __forceinline__ float mlp_forward16(const MlpFrags& F, v4s x0, v4s x1, MlpFwdState* st) {
  v4f d1[2], d2[2];
  v4s h[2];
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    v4f c = {0.f, 0.f, 0.f, 0.f};
    c = mfma16(F.a1[nb][0], x0, c);
    c = mfma16(F.a1[nb][1], x1, c);
    d1[nb] = c;
    float hv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) hv[i] = fmaxf(c[i] + F.b1[nb][i], 0.f);
    h[nb] = pack4(hv[0], hv[1], hv[2], hv[3]);
  }
  float part = 0.f;
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    v4f c = {0.f, 0.f, 0.f, 0.f};
    c = mfma16(F.a2[nb][0], h[0], c);
    c = mfma16(F.a2[nb][1], h[1], c);
    d2[nb] = c;
#pragma unroll
    for (int i = 0; i < 4; ++i) part += F.w3[nb][i] * fmaxf(c[i] + F.b2[nb][i], 0.f);
  }
  part += __shfl_xor(part, 16);
  part += __shfl_xor(part, 32);
  if (st) {
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) { st->a1[nb] = d1[nb]; st->a2[nb] = d2[nb]; st->h[nb] = h[nb]; }
  }
  return part + F.b3;
}

// ---------------------------------------------------------------------------
// Features and plain labels of a whole grid (training data, evaluation), for
// both directions: rows [0, n) are the evaluations along x, rows [n, 2n) those
// along y (the same four stencil groups, y-groups first).
struct MlpFeatParams {
  const double* Q;
  unsigned short* feat;   // [2][n][32]
  uint8_t* chi;           // [2][n] or null: plain labels [psi_x < psi_c], [psi_y < psi_c]
  int nx, ny, bcx, bcy;
  double gamma;
};

__device__ __forceinline__ int wrap_bc(int k, int n, int bc) {
  if (bc == 0) {
    while (k < 0) k += n;
    while (k >= n) k -= n;
    return k;
  }
  return k < 0 ? 0 : (k >= n ? n - 1 : k);
}

// Pressure of a cell as the features define it: u = (rho u)/rho and v by
// IEEE division, p = (gamma-1) (E - rho (u u + v v) / 2), every product and
// sum rounded on its own.  The two quotients share one refined reciprocal
// (div_rb: the IEEE quotient bit for bit inside its operand range).
__device__ __forceinline__ double mlp_cell_pressure(double r, double mx, double my, double E,
                                                    double gamma) {
#pragma clang fp contract(off)
  double u, v;
  if (r != 0.0 && div_rb_ok(r) && div_rb_ok(mx) && div_rb_ok(my)) {
    const double rb = rcp_nr(r);
    u = div_rb(mx, r, rb);
    v = div_rb(my, r, rb);
  } else {
    u = mx / r;
    v = my / r;
  }
  return (gamma - 1.0) * (E - r * (u * u + v * v) / 2.0);
}

__global__ __launch_bounds__(256) void mlp_features_kernel(MlpFeatParams P) {
  const size_t n = (size_t)P.nx * P.ny;
  const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int i = (int)(c / P.nx), j = (int)(c % P.nx);
  auto cell = [&](int ii, int jj, int want_p) -> double {
    const size_t s = (size_t)wrap_bc(ii, P.ny, P.bcy) * P.nx + wrap_bc(jj, P.nx, P.bcx);
    const double r = P.Q[s];
    if (!want_p) return r;
    return mlp_cell_pressure(r, P.Q[n + s], P.Q[2 * n + s], P.Q[3 * n + s], P.gamma);
  };
  unsigned f[kMlpIn / 2];
  mlp_cell_features(
      [&](int s, int o) {
        return (s < 2) ? cell(i, j + o, s & 1) : cell(i + o, j, s & 1);
      },
      f);
  uint4* dx = reinterpret_cast<uint4*>(P.feat + c * kMlpIn);
  uint4* dy = reinterpret_cast<uint4*>(P.feat + (n + c) * kMlpIn);
  unsigned fy[kMlpIn / 2];
#pragma unroll
  for (int k = 0; k < kMlpF / 2; ++k) fy[k] = f[(k + kMlpF / 4) % (kMlpF / 2)];
  fy[kMlpF / 2] = 0;
  fy[kMlpF / 2 + 1] = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    dx[q] = make_uint4(f[4 * q], f[4 * q + 1], f[4 * q + 2], f[4 * q + 3]);
    dy[q] = make_uint4(fy[4 * q], fy[4 * q + 1], fy[4 * q + 2], fy[4 * q + 3]);
  }
  if (P.chi) {
    const double px = detector_psi(cell(i, j - 2, 0), cell(i, j - 1, 0), cell(i, j, 0),
                                   cell(i, j + 1, 0), cell(i, j + 2, 0));
    const double py = detector_psi(cell(i - 2, j, 0), cell(i - 1, j, 0), cell(i, j, 0),
                                   cell(i + 1, j, 0), cell(i + 2, j, 0));
    P.chi[c] = px < kPsiC ? 1 : 0;
    P.chi[n + c] = py < kPsiC ? 1 : 0;
  }
}

// ---------------------------------------------------------------------------
// Per-cell flag map of the learned detector, chi[c] for every grid cell:
// bit 0 from the evaluation along x, bit 1 from the one along y, each the
// logit's sign where |logit| >= margin, else the plain label
// [psi^d < psi_c] from the FP64 density.  One workgroup per
// 64 x 16 block of cells: the block plus a 3-cell halo of rho and p (float32)
// is staged in LDS once (ghost cells by wrap or clamp), then four
// rounds of 256 cells each compute their features (one cell per thread),
// stage them as bf16 rows and run the network on the matrix cores; a wave
// evaluates exactly its own 64 cells, so the logit of lane l's cell lands in
// lane l.  Evaluations below the margin are queued per wave and settled after
// the last round; the flag bytes are then stored coalesced, one row per wave.
struct MlpChiParams {
  const double* Q;
  // optional: rho and p of Q already rounded to float32, [2][ny][nx] (the
  // values the block staging computes from Q; written beside Q by the
  // stage that produced it), read instead of Q
  const float* rp;
  uint8_t* chi;                 // [ny][nx]: bit 0 chi^x, bit 1 chi^y
  unsigned long long* nfb;      // plain fallbacks (summed over both directions)
  MlpImage M;
  float margin;
  int nx, ny, bcx, bcy, tiles_x;
  double gamma;
};
#ifndef GBR_CHI_TY
#define GBR_CHI_TY 16
#endif
constexpr int kChiTX = 64, kChiTY = GBR_CHI_TY;
constexpr int kChiRX = kChiTX + 6, kChiRY = kChiTY + 6, kChiRS = kChiRX * kChiRY;
constexpr int kChiRow = 5;            // uint4 per staged feature row (80 B: conflict-free)

__global__ __launch_bounds__(256, 4) void mlp_chi_kernel(MlpChiParams P) {
  constexpr int NC = kChiTX * kChiTY;          // cells of the block
  constexpr int QW = 2 * 64 * (kChiTY / 4);    // fallback entries a wave can queue
  __shared__ float sF[2][kChiRS];
  __shared__ uint4 sX[256 * kChiRow];
  __shared__ unsigned char sCx[NC], sCy[NC];   // per-cell bit along x, along y
  __shared__ unsigned short sQ[4][QW];         // per wave: 2 cell + direction
  __shared__ unsigned sFb[4];
  const int tid = threadIdx.x, l = __lane_id(), g = l >> 4, w = tid >> 6;
  // workgroups are dealt to the 8 XCDs round-robin: give each XCD one
  // contiguous run of blocks, so neighbouring blocks share halo rows in its L2
  const int xcd = blockIdx.x & 7, per = gridDim.x >> 3, rem = gridDim.x & 7;
  const int blk = xcd * per + (xcd < rem ? xcd : rem) + (blockIdx.x >> 3);
  const int tx0 = (blk % P.tiles_x) * kChiTX, ty0 = (blk / P.tiles_x) * kChiTY;
  const size_t n = (size_t)P.nx * P.ny;
  constexpr int LR = (kChiRS + 255) / 256;
  // ghost cells: on grids of at least one block plus halo a single wrap (or
  // a clamp) suffices; smaller grids take the general loop
  const bool one = P.nx >= kChiRX && P.ny >= kChiRY;
  auto gwrap = [&](int k, int nn, int bc) {
    if (!one) return wrap_bc(k, nn, bc);
    if (bc != 0) return min(max(k, 0), nn - 1);
    k = k < 0 ? k + nn : k;
    return k >= nn ? k - nn : k;
  };
  // the network's fragments first: their loads overlap those of the state
  MlpInfer F;
  mlp_load_infer(P.M, F);
  auto src = [&](int c) {
    return (size_t)gwrap(ty0 + c / kChiRX - 3, P.ny, P.bcy) * P.nx +
           gwrap(tx0 + c % kChiRX - 3, P.nx, P.bcx);
  };
  if (P.rp) {
    float q[LR][2];
#pragma unroll
    for (int k = 0; k < LR; ++k) {
      const int c = tid + 256 * k;
      if (c < kChiRS) {
        const size_t s = src(c);
        q[k][0] = P.rp[s];
        q[k][1] = P.rp[n + s];
      }
    }
#pragma unroll
    for (int k = 0; k < LR; ++k) {
      const int c = tid + 256 * k;
      if (c < kChiRS) {
        sF[0][c] = q[k][0];
        sF[1][c] = q[k][1];
      }
    }
  } else {
    double q[LR][4];
#pragma unroll
    for (int k = 0; k < LR; ++k) {
      const int c = tid + 256 * k;
      if (c < kChiRS) {
        const size_t s = src(c);
#pragma unroll
        for (int m = 0; m < 4; ++m) q[k][m] = P.Q[m * n + s];
      }
    }
#pragma unroll
    for (int k = 0; k < LR; ++k) {
      const int c = tid + 256 * k;
      if (c < kChiRS) {
        sF[0][c] = (float)q[k][0];
        sF[1][c] = (float)mlp_cell_pressure(q[k][0], q[k][1], q[k][2], q[k][3], P.gamma);
      }
    }
  }
  __syncthreads();
  // Wave w evaluates rows 4 rnd + w; it stages and reads back only its own 64
  // feature rows, and queues and settles only its own fallbacks, so every
  // hand-off needs a wave-scope fence, not a barrier.
  int nq = 0;   // the wave's queued fallbacks (uniform across the wave)
  for (int rnd = 0; rnd < kChiTY / 4; ++rnd) {
    const int lx = tid & 63, ly = 4 * rnd + w;
    const int rc = (ly + 3) * kChiRX + lx + 3;
    {
      unsigned f[kMlpIn / 2];
      mlp_cell_features(
          [&](int s, int o) { return sF[s & 1][rc + o * ((s < 2) ? 1 : kChiRX)]; }, f);
#pragma unroll
      for (int c4 = 0; c4 < 4; ++c4)
        sX[tid * kChiRow + c4] = make_uint4(f[4 * c4], f[4 * c4 + 1], f[4 * c4 + 2], f[4 * c4 + 3]);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    float zx = 0.f, zy = 0.f;
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      const v8s v = __builtin_bit_cast(v8s, sX[(w * 64 + cb * 16 + (l & 15)) * kChiRow + g]);
      const float z0 = mlp_infer16(F, v, false);
      const float z1 = mlp_infer16(F, v, true);
      if (cb == g) { zx = z0; zy = z1; }
    }
    // the network's sign where |logit| >= margin; below it the plain label
    // along that direction, settled after the last round
    const int cell = ly * kChiTX + lx;
    const bool inb = tx0 + lx < P.nx && ty0 + ly < P.ny;
    const bool fx = inb && !(fabsf(zx) >= P.margin);
    const bool fy = inb && !(fabsf(zy) >= P.margin);
    sCx[cell] = (!fx && zx > 0.f) ? 1 : 0;
    sCy[cell] = (!fy && zy > 0.f) ? 2 : 0;
    const unsigned long long bx = __ballot(fx), by = __ballot(fy);
    const unsigned long long below = (1ull << l) - 1ull;
    if (fx) sQ[w][nq + (int)__popcll(bx & below)] = (unsigned short)(2 * cell);
    nq += (int)__popcll(bx);
    if (fy) sQ[w][nq + (int)__popcll(by & below)] = (unsigned short)(2 * cell + 1);
    nq += (int)__popcll(by);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  // plain labels of the queued evaluations, one per lane, from the FP64
  // density in memory
  for (int k = l; k < nq; k += 64) {
    const int e = sQ[w][k], cell = e >> 1, ydir = e & 1;
    const int gi = ty0 + cell / kChiTX, gj = tx0 + cell % kChiTX;
    const int si = ydir, sj = 1 - ydir;
    auto rho = [&](int o) {
      return P.Q[(size_t)gwrap(gi + o * si, P.ny, P.bcy) * P.nx + gwrap(gj + o * sj, P.nx, P.bcx)];
    };
    if (detector_flag(rho(-2), rho(-1), rho(0), rho(1), rho(2))) {
      if (ydir) sCy[cell] = 2; else sCx[cell] = 1;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  for (int rnd = 0; rnd < kChiTY / 4; ++rnd) {
    const int lx = tid & 63, ly = 4 * rnd + w;
    const int gj = tx0 + lx, gi = ty0 + ly;
    const int cell = ly * kChiTX + lx;
    if (gj < P.nx && gi < P.ny) P.chi[(size_t)gi * P.nx + gj] = (uint8_t)(sCx[cell] | sCy[cell]);
  }
  if (P.nfb) {
    if (l == 0) sFb[w] = (unsigned)nq;
    __syncthreads();
    if (tid == 0) {
      const unsigned t = (sFb[0] + sFb[1]) + (sFb[2] + sFb[3]);
      if (t) atomicAdd(P.nfb, (unsigned long long)t);
    }
  }
}

// ---------------------------------------------------------------------------
// Inference over a feature array: logits[c] for c < n.  One wave per 64 cells.
__global__ __launch_bounds__(256) void mlp_forward_kernel(MlpImage M, const unsigned short* feat,
                                                          int n, float* logits) {
  MlpInfer F;
  mlp_load_infer(M, F);
  const int l = __lane_id(), r = l & 15, g = l >> 4;
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    const int c = wave * 64 + cb * 16 + r;
    const int cc = c < n ? c : n - 1;
    const v8s x = *reinterpret_cast<const v8s*>(feat + (size_t)cc * kMlpIn + 8 * g);
    const float z = mlp_infer16(F, x);
    if (g == 0 && c < n) logits[c] = z;
  }
}

// ---------------------------------------------------------------------------
// Training: per workgroup of 256 threads, 256 batch cells (64 per wave):
// forward, BCE-with-logits loss, backward; the workgroup's gradient sum is
// written to partial[blockIdx.x][0..2016] and its loss sum to [2017].
struct MlpGradParams {
  MlpImage M;
  const unsigned short* feat;   // [N][32]
  const uint8_t* label;         // [N]
  const int* idx;               // [batch]
  int batch;
  float* partial;               // [nblocks][kMlpNP + 1]
};

__global__ __launch_bounds__(256) void mlp_grad_kernel(MlpGradParams P) {
  __shared__ unsigned short sT[4][2][16 * kMlpIn];   // per wave: [0] dh rows, [1] activation rows
  __shared__ float sRed[4][kMlpNP + 1];
  const int l = __lane_id(), r = l & 15, g = l >> 4, w = threadIdx.x >> 6;
  MlpFrags F;
  mlp_load_frags(P.M, F);
  // A operand of dh1^T = W2^T dh2^T: lane holds W2[16 ks + 4 g + i][16 mb + r]
  v4s a2t[2][2];
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        a2t[mb][ks][i] = (short)P.M.W2[(16 * ks + 4 * g + i) * kMlpH + 16 * mb + r];
  const float invB = 1.0f / (float)P.batch;

  v4f gW1[2][2], gW2[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      gW1[a][b] = (v4f){0.f, 0.f, 0.f, 0.f};
      gW2[a][b] = (v4f){0.f, 0.f, 0.f, 0.f};
    }
  float gw3[2][4], gb1[2][4], gb2[2][4], gb3 = 0.f, lsum = 0.f;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int i = 0; i < 4; ++i) { gw3[a][i] = 0.f; gb1[a][i] = 0.f; gb2[a][i] = 0.f; }

  unsigned short* sDh = sT[w][0];
  unsigned short* sAct = sT[w][1];
#pragma unroll 1
  for (int cb = 0; cb < 4; ++cb) {
    const int bi = blockIdx.x * 256 + w * 64 + cb * 16 + r;
    const bool valid = bi < P.batch;
    const int cell = P.idx[valid ? bi : 0];
    const unsigned short* xr = P.feat + (size_t)cell * kMlpIn;
    const v4s x0 = *reinterpret_cast<const v4s*>(xr + 4 * g);
    const v4s x1 = *reinterpret_cast<const v4s*>(xr + 16 + 4 * g);
    MlpFwdState st;
    const float z = mlp_forward16(F, x0, x1, &st);
    const float y = valid ? (float)P.label[cell] : 0.f;
    // mean BCE with logits; dz = (sigmoid(z) - y) / B
    const float dz = valid ? (1.0f / (1.0f + __expf(-z)) - y) * invB : 0.f;
    if (g == 0 && valid) lsum += fmaxf(z, 0.f) - z * y + __logf(1.0f + __expf(-fabsf(z)));
    // output layer and dh2 (D layout: lane holds neurons 16 nb + 4 g + i of cell r)
    float dh2[2][4];
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float a2 = st.a2[nb][i] + F.b2[nb][i];
        const float h2 = fmaxf(a2, 0.f);
        gw3[nb][i] += dz * h2;
        dh2[nb][i] = (a2 > 0.f) ? dz * F.w3[nb][i] : 0.f;
        gb2[nb][i] += dh2[nb][i];
      }
    gb3 += (g == 0) ? dz : 0.f;
    v4s dh2p[2];
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) dh2p[nb] = pack4(dh2[nb][0], dh2[nb][1], dh2[nb][2], dh2[nb][3]);
    // dh1^T = W2^T dh2^T, masked by the layer-1 activation
    v4s dh1p[2];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
      v4f c = {0.f, 0.f, 0.f, 0.f};
      c = mfma16(a2t[mb][0], dh2p[0], c);
      c = mfma16(a2t[mb][1], dh2p[1], c);
      float d[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        d[i] = (st.a1[mb][i] + F.b1[mb][i] > 0.f) ? c[i] : 0.f;
        gb1[mb][i] += d[i];
      }
      dh1p[mb] = pack4(d[0], d[1], d[2], d[3]);
    }
    // weight gradients need the cells as the reduction dimension: stage the
    // 16-cell blocks of dh2 and h1 (then dh1 and x) row-wise in LDS and read
    // them back transposed.
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        sDh[r * kMlpIn + 16 * nb + 4 * g + i] = (unsigned short)dh2p[nb][i];
        sAct[r * kMlpIn + 16 * nb + 4 * g + i] = (unsigned short)st.h[nb][i];
      }
    __syncthreads();
    // dW2[n2][k] += sum_c dh2[c][n2] h1[c][k]: A = dh2^T, B = h1 (K = cells)
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
      v4s a;
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = (short)sDh[(4 * g + i) * kMlpIn + 16 * mb + r];
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) {
        v4s b;
#pragma unroll
        for (int i = 0; i < 4; ++i) b[i] = (short)sAct[(4 * g + i) * kMlpIn + 16 * nb + r];
        gW2[mb][nb] = mfma16(a, b, gW2[mb][nb]);
      }
    }
    __syncthreads();
    // dW1[n1][k] += sum_c dh1[c][n1] x[c][k]
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int i = 0; i < 4; ++i) sDh[r * kMlpIn + 16 * mb + 4 * g + i] = (unsigned short)dh1p[mb][i];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      sAct[r * kMlpIn + 4 * g + i] = (unsigned short)x0[i];
      sAct[r * kMlpIn + 16 + 4 * g + i] = (unsigned short)x1[i];
    }
    __syncthreads();
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
      v4s a;
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = (short)sDh[(4 * g + i) * kMlpIn + 16 * mb + r];
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) {
        v4s b;
#pragma unroll
        for (int i = 0; i < 4; ++i) b[i] = (short)sAct[(4 * g + i) * kMlpIn + 16 * nb + r];
        gW1[mb][nb] = mfma16(a, b, gW1[mb][nb]);
      }
    }
    __syncthreads();
  }
  // reduce the per-lane partial sums over the 16 cells of each lane column
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) {
        gw3[a][i] += __shfl_xor(gw3[a][i], o);
        gb1[a][i] += __shfl_xor(gb1[a][i], o);
        gb2[a][i] += __shfl_xor(gb2[a][i], o);
      }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    gb3 += __shfl_xor(gb3, o);
    lsum += __shfl_xor(lsum, o);
  }
  float* red = sRed[w];
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = 16 * mb + 4 * g + i, col = 16 * nb + r;
        if (col < kMlpF) red[row * kMlpF + col] = gW1[mb][nb][i];
        red[kMlpH * kMlpF + row * kMlpH + col] = gW2[mb][nb][i];
      }
  if (r == 0) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int nn = 16 * a + 4 * g + i;
        red[kMlpH * kMlpF + kMlpH * kMlpH + nn] = gw3[a][i];
        red[kMlpNW + nn] = gb1[a][i];
        red[kMlpNW + kMlpH + nn] = gb2[a][i];
      }
  }
  if (l == 0) {
    red[kMlpNW + 2 * kMlpH] = gb3;
    red[kMlpNP] = lsum;
  }
  __syncthreads();
  for (int p = threadIdx.x; p < kMlpNP + 1; p += 256)
    P.partial[(size_t)blockIdx.x * (kMlpNP + 1) + p] =
        ((sRed[0][p] + sRed[1][p]) + sRed[2][p]) + sRed[3][p];
}

// Sum of the workgroup partials in a fixed order: grad[p] (and loss at kMlpNP).
__global__ __launch_bounds__(256) void mlp_sum_kernel(const float* partial, int nblk, float* out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > kMlpNP) return;
  float s = 0.f;
  for (int b = 0; b < nblk; ++b) s += partial[(size_t)b * (kMlpNP + 1) + p];
  out[p] = s;
}

// Adam step on the float32 master parameters [2017] (weights then biases) and
// refresh of the bf16 inference image.
struct AdamParams {
  const float* grad;   // [kMlpNP + 1]
  float* master;       // [kMlpNP]
  float* m;
  float* v;
  unsigned short* W1;  // [32][32]
  unsigned short* W2;  // [32][32]
  float* w3;           // [32]
  float* b;            // [65]
  float lr, beta1, beta2, eps, bc1, bc2;   // bc = 1 - beta^t
};

__device__ __forceinline__ void mlp_publish(int p, float w, unsigned short* W1, unsigned short* W2,
                                            float* w3, float* b) {
  if (p < kMlpH * kMlpF) {
    W1[(p / kMlpF) * kMlpIn + p % kMlpF] = f2bf(w);
  } else if (p < kMlpH * kMlpF + kMlpH * kMlpH) {
    W2[p - kMlpH * kMlpF] = f2bf(w);
  } else if (p < kMlpNW) {
    w3[p - kMlpH * kMlpF - kMlpH * kMlpH] = bf2f(f2bf(w));
  } else {
    b[p - kMlpNW] = w;
  }
}

__global__ __launch_bounds__(256) void mlp_adam_kernel(AdamParams A) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kMlpNP) return;
  const float gr = A.grad[p];
  const float m = A.beta1 * A.m[p] + (1.f - A.beta1) * gr;
  const float v = A.beta2 * A.v[p] + (1.f - A.beta2) * gr * gr;
  A.m[p] = m;
  A.v[p] = v;
  const float w = A.master[p] - A.lr * (m / A.bc1) / (sqrtf(v / A.bc2) + A.eps);
  A.master[p] = w;
  mlp_publish(p, w, A.W1, A.W2, A.w3, A.b);
}

// Publish a full parameter vector (after a host upload): zero the padding too.
__global__ __launch_bounds__(256) void mlp_publish_kernel(const float* master, unsigned short* W1,
                                                          unsigned short* W2, float* w3, float* b) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < kMlpH * (kMlpIn - kMlpF)) W1[(p / (kMlpIn - kMlpF)) * kMlpIn + kMlpF + p % (kMlpIn - kMlpF)] = 0;
  if (p < kMlpNP) mlp_publish(p, master[p], W1, W2, w3, b);
}

// Exhaustive check of rcp_rn against IEEE division over the floats with bit
// patterns in [lo, hi): mismatches are counted in *count.
__global__ __launch_bounds__(256) void rcp_selftest_kernel(unsigned lo, unsigned hi,
                                                           unsigned long long* count) {
  const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
  unsigned long long bad = 0;
  for (unsigned long long b = lo + (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; b < hi;
       b += stride) {
    const float x = __uint_as_float((unsigned)b);
    if (__float_as_uint(rcp_rn(x)) != __float_as_uint(1.0f / x)) ++bad;
  }
  if (bad) atomicAdd(count, bad);
}

}  // namespace gbr
