// Learned per-edge cost model: a 16-64-64-1 multilayer perceptron with ReLU,
// bf16 weights and fp32 accumulation, trained on the GPU by the kernels below
// (forward, backward, fixed-order gradient reduction, Adam), and used to order
// and bin edges for the counting kernels.  Counts never depend on it.
//
// Parameter layout (fp32 master copy, NPARAM floats):
//   W1[64][16], b1[64], W2[64][64], b2[64], w3[64], b3[1]
// Features per edge (i, j), d_lo <= d_hi the endpoint degrees, c[t] the type
// histogram of the common neighbours (tau_e[t] / |T_ij|, known before any
// per-edge counting) and h[t] the combined neighbour type histogram
// (D[i][t] + D[j][t]) / (d_i + d_j), types >= 8 folded onto t mod 8:
//   0 log2(1+d_lo)  1 log2(1+d_hi)  2 log2(1+d_lo*d_hi)  3 [phi_i == phi_j]
//   4..11 c[0..7]  12 log2(1 + |T_ij|)  13 entropy of h (bits)
//   14 h[phi_i]  15 h[phi_j]
// Features are standardised with the training sample's mean and deviation.
// Target: log2(1 + work), work = the instrumented element-visit count of the
// per-edge counting kernel for that edge.

#include "tg_device.h"

namespace tg {

#define TG_MLP_IN 16
#define TG_MLP_H 64
#define TG_MLP_NPARAM (TG_MLP_H * TG_MLP_IN + TG_MLP_H + TG_MLP_H * TG_MLP_H + TG_MLP_H + TG_MLP_H + 1)
#define TG_MLP_OFF_B1 (TG_MLP_H * TG_MLP_IN)
#define TG_MLP_OFF_W2 (TG_MLP_OFF_B1 + TG_MLP_H)
#define TG_MLP_OFF_B2 (TG_MLP_OFF_W2 + TG_MLP_H * TG_MLP_H)
#define TG_MLP_OFF_W3 (TG_MLP_OFF_B2 + TG_MLP_H)
#define TG_MLP_OFF_B3 (TG_MLP_OFF_W3 + TG_MLP_H)
#define TG_MLP_ROWS 32   // rows per workgroup in the training kernel

// Round-to-nearest-even fp32 -> bf16, kept as fp32 value.
__device__ __host__ __forceinline__ float bf16_round(float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  if ((u & 0x7F800000u) == 0x7F800000u) return x;  // inf / nan unchanged
  const uint32_t lsb = (u >> 16) & 1u;
  u = (u + 0x7FFFu + lsb) & 0xFFFF0000u;
  float r;
  memcpy(&r, &u, 4);
  return r;
}

// ------------------------------------------------------------- features --

__device__ __forceinline__ void edge_features(int32_t e, int32_t i, int32_t j, const int32_t* deg,
                                              const uint32_t* D, const uint32_t* tau, const uint8_t* ty, int L,
                                              float f[TG_MLP_IN]) {
  const float di = (float)deg[i], dj = (float)deg[j];
  const float lo = fminf(di, dj), hi = fmaxf(di, dj);
  float h[8] = {0, 0, 0, 0, 0, 0, 0, 0}, c[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  float nT = 0.0f;
  const float tot = di + dj;
  for (int t = 0; t < L; ++t) {
    h[t & 7] += (float)(D[(int64_t)i * L + t] + D[(int64_t)j * L + t]);
    const float ct = (float)tau[(int64_t)e * L + t];
    c[t & 7] += ct;
    nT += ct;
  }
  float ent = 0.0f;
  for (int t = 0; t < 8; ++t) {
    h[t] = tot > 0 ? h[t] / tot : 0.0f;
    c[t] = nT > 0 ? c[t] / nT : 0.0f;
    if (h[t] > 0) ent -= h[t] * log2f(h[t]);
  }
  f[0] = log2f(1.0f + lo);
  f[1] = log2f(1.0f + hi);
  f[2] = log2f(1.0f + lo * hi);
  f[3] = ty[i] == ty[j] ? 1.0f : 0.0f;
  for (int t = 0; t < 8; ++t) f[4 + t] = c[t];
  f[12] = log2f(1.0f + nT);
  f[13] = ent;
  f[14] = h[ty[i] & 7];
  f[15] = h[ty[j] & 7];
}

// Features of the listed edges (list null: edges 0..count-1).
__global__ void k_mlp_features(int64_t count, const int32_t* __restrict__ list, const int32_t* __restrict__ ei,
                               const int32_t* __restrict__ ej, const int32_t* __restrict__ deg,
                               const uint32_t* __restrict__ D, const uint32_t* __restrict__ tau,
                               const uint8_t* __restrict__ ty, int L, float* __restrict__ X) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < count; q += (int64_t)gridDim.x * blockDim.x) {
    const int32_t e = list ? list[q] : (int32_t)q;
    float f[TG_MLP_IN];
    edge_features(e, ei[e], ej[e], deg, D, tau, ty, L, f);
    for (int c = 0; c < TG_MLP_IN; ++c) X[q * TG_MLP_IN + c] = f[c];
  }
}

// Mean and standard deviation of each feature column (one workgroup, fixed
// summation order).  stats[0..16) mean, stats[16..32) deviation (>= 1e-3).
__global__ void k_mlp_feature_stats(int64_t n, const float* __restrict__ X, float* __restrict__ stats) {
  const int c0 = (threadIdx.x & 3) * 4;   // four threads per row group share the 16 columns
  const int r0 = threadIdx.x >> 2;        // 64 row lanes
  double a[4] = {0, 0, 0, 0}, b[4] = {0, 0, 0, 0};
  for (int64_t r = r0; r < n; r += 64)
    for (int q = 0; q < 4; ++q) {
      const double x = X[r * TG_MLP_IN + c0 + q];
      a[q] += x;
      b[q] += x * x;
    }
  __shared__ double sa[64][TG_MLP_IN], sb[64][TG_MLP_IN];
  for (int q = 0; q < 4; ++q) { sa[r0][c0 + q] = a[q]; sb[r0][c0 + q] = b[q]; }
  __syncthreads();
  if (threadIdx.x < TG_MLP_IN) {
    double A = 0, B = 0;
    for (int r = 0; r < 64; ++r) { A += sa[r][threadIdx.x]; B += sb[r][threadIdx.x]; }
    const double mean = n > 0 ? A / (double)n : 0.0;
    const double var = n > 0 ? fmax(B / (double)n - mean * mean, 0.0) : 1.0;
    stats[threadIdx.x] = (float)mean;
    stats[TG_MLP_IN + threadIdx.x] = (float)fmax(sqrt(var), 1e-3);
  }
}

// --------------------------------------------------------------- forward --

// Forward pass of one standardised row with bf16 weights held in LDS as fp32.
__device__ __forceinline__ float mlp_forward_row(const float* __restrict__ P, const float* x, float* h1, float* h2) {
  for (int a = 0; a < TG_MLP_H; ++a) {
    float s = P[TG_MLP_OFF_B1 + a];
#pragma unroll
    for (int c = 0; c < TG_MLP_IN; ++c) s = fmaf(P[a * TG_MLP_IN + c], x[c], s);
    h1[a] = fmaxf(s, 0.0f);
  }
  float y = P[TG_MLP_OFF_B3];
  for (int a = 0; a < TG_MLP_H; ++a) {
    float s = P[TG_MLP_OFF_B2 + a];
    for (int b = 0; b < TG_MLP_H; ++b) s = fmaf(P[TG_MLP_OFF_W2 + a * TG_MLP_H + b], h1[b], s);
    h2[a] = fmaxf(s, 0.0f);
    y = fmaf(P[TG_MLP_OFF_W3 + a], h2[a], y);
  }
  return y;
}

__device__ __forceinline__ void load_params_bf16(const uint16_t* __restrict__ Pbf, float* P) {
  for (int q = threadIdx.x; q < TG_MLP_NPARAM; q += blockDim.x) {
    const uint32_t u = (uint32_t)Pbf[q] << 16;
    float f;
    memcpy(&f, &u, 4);
    P[q] = f;
  }
}

// Predicted log2 cost of the rows of X (or of edges 0..count-1 when X is
// null: features are then computed from the graph), on bf16 matrix cores.
// One wavefront takes 16 rows at a time: layer 1 is [16 x 16] x [16 x 64]
// (four 16x16x16 MFMAs), layer 2 [16 x 64] x [64 x 64] (sixteen), with the
// standardised inputs and the first hidden layer rounded to bf16 (weights are
// bf16 already) and fp32 accumulation; layer 3 is a dot product on the vector
// ALUs.  Operand layouts of v_mfma_f32_16x16x16_bf16, lane l, r = l % 16,
// g = l / 16: A holds A[r][4g .. 4g+3], B holds B[4g .. 4g+3][r], and the
// result holds D[4g .. 4g+3][r].
typedef __attribute__((__vector_size__(4 * sizeof(short)))) short tg_bf16x4;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float tg_f32x4;

__device__ __forceinline__ short bf16_bits(float x) {
  const float r = bf16_round(x);
  uint32_t u;
  memcpy(&u, &r, 4);
  return (short)(u >> 16);
}

__device__ __forceinline__ float bf16_value(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}

__global__ void __launch_bounds__(256) k_mlp_predict(int64_t count, const uint16_t* __restrict__ Pbf,
                                                     const float* __restrict__ stats, const float* __restrict__ X,
                                                     const int32_t* __restrict__ ei, const int32_t* __restrict__ ej,
                                                     const int32_t* __restrict__ deg, const uint32_t* __restrict__ D,
                                                     const uint32_t* __restrict__ tau, const uint8_t* __restrict__ ty,
                                                     int L, float* __restrict__ out) {
  __shared__ short hbuf[4][16 * TG_MLP_H];  // per wavefront: first hidden layer, bf16, row-major
  const int wib = threadIdx.x / TG_WAVE, l = lane();
  const int r = l & 15, g = l >> 4;
  tg_bf16x4 B1[4], B2[4][4];
  float b1v[4], b2v[4], w3v[4];
  for (int nt = 0; nt < 4; ++nt) {
    const int n = nt * 16 + r;
    for (int j = 0; j < 4; ++j) B1[nt][j] = (short)Pbf[n * TG_MLP_IN + 4 * g + j];
    for (int ks = 0; ks < 4; ++ks)
      for (int j = 0; j < 4; ++j) B2[ks][nt][j] = (short)Pbf[TG_MLP_OFF_W2 + n * TG_MLP_H + ks * 16 + 4 * g + j];
    b1v[nt] = bf16_value(Pbf[TG_MLP_OFF_B1 + n]);
    b2v[nt] = bf16_value(Pbf[TG_MLP_OFF_B2 + n]);
    w3v[nt] = bf16_value(Pbf[TG_MLP_OFF_W3 + n]);
  }
  const float b3 = bf16_value(Pbf[TG_MLP_OFF_B3]);
  float mean[4], inv[4];
  for (int j = 0; j < 4; ++j) {
    mean[j] = stats[4 * g + j];
    inv[j] = 1.0f / stats[TG_MLP_IN + 4 * g + j];
  }
  short* hb = hbuf[wib];
  for (int64_t tile = (int64_t)blockIdx.x * 4 + wib; tile * 16 < count; tile += (int64_t)gridDim.x * 4) {
    const int64_t row = tile * 16 + r;
    float f[TG_MLP_IN];
    if (row < count) {
      if (X) {
        for (int c = 0; c < TG_MLP_IN; ++c) f[c] = X[row * TG_MLP_IN + c];
      } else {
        edge_features((int32_t)row, ei[row], ej[row], deg, D, tau, ty, L, f);
      }
    } else {
      for (int c = 0; c < TG_MLP_IN; ++c) f[c] = 0.0f;
    }
    tg_bf16x4 a;
    for (int j = 0; j < 4; ++j) a[j] = bf16_bits((f[4 * g + j] - mean[j]) * inv[j]);
    // layer 1, bias, ReLU, bf16 into LDS
    for (int nt = 0; nt < 4; ++nt) {
      tg_f32x4 h = {0.0f, 0.0f, 0.0f, 0.0f};
      h = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, B1[nt], h, 0, 0, 0);
      for (int j = 0; j < 4; ++j) hb[(4 * g + j) * TG_MLP_H + nt * 16 + r] = bf16_bits(fmaxf(h[j] + b1v[nt], 0.0f));
    }
    wave_sync();
    // layer 2
    tg_f32x4 o[4];
    for (int nt = 0; nt < 4; ++nt) o[nt] = (tg_f32x4){0.0f, 0.0f, 0.0f, 0.0f};
    for (int ks = 0; ks < 4; ++ks) {
      tg_bf16x4 a2;
      for (int j = 0; j < 4; ++j) a2[j] = hb[r * TG_MLP_H + ks * 16 + 4 * g + j];
      for (int nt = 0; nt < 4; ++nt) o[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a2, B2[ks][nt], o[nt], 0, 0, 0);
    }
    wave_sync();
    // layer 3: rows 4g .. 4g+3, column r of each tile, summed over the 16
    // lanes of the group
    float part[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int nt = 0; nt < 4; ++nt)
      for (int j = 0; j < 4; ++j) part[j] = fmaf(w3v[nt], fmaxf(o[nt][j] + b2v[nt], 0.0f), part[j]);
    for (int off = 1; off < 16; off <<= 1)
      for (int j = 0; j < 4; ++j) part[j] += __shfl_xor(part[j], off, TG_WAVE);
    if (r == 0)
      for (int j = 0; j < 4; ++j) {
        const int64_t orow = tile * 16 + 4 * g + j;
        if (orow < count) out[orow] = part[j] + b3;
      }
  }
}

// -------------------------------------------------------------- backward --

// One workgroup per TG_MLP_ROWS rows of a mini-batch: forward, MSE loss
// gradient (mean over the whole mini-batch of `total` rows), backward, and a
// per-workgroup partial gradient written to partial[blockIdx.x][NPARAM]
// together with the partial loss in partial_loss[blockIdx.x].
__global__ void __launch_bounds__(256) k_mlp_backward(int64_t nrows, int64_t total, const int32_t* __restrict__ rows,
                                                      const uint16_t* __restrict__ Pbf,
                                                      const float* __restrict__ stats, const float* __restrict__ X,
                                                      const float* __restrict__ Y, float* __restrict__ partial,
                                                      float* __restrict__ partial_loss) {
  __shared__ float P[TG_MLP_NPARAM];
  __shared__ float xs[TG_MLP_ROWS][TG_MLP_IN];
  __shared__ float h1s[TG_MLP_ROWS][TG_MLP_H];
  __shared__ float d2s[TG_MLP_ROWS][TG_MLP_H];   // delta at layer-2 pre-activations
  __shared__ float d1s[TG_MLP_ROWS][TG_MLP_H];   // delta at layer-1 pre-activations
  __shared__ float dys[TG_MLP_ROWS];
  __shared__ float h2s[TG_MLP_ROWS][TG_MLP_H];
  load_params_bf16(Pbf, P);
  __syncthreads();
  const int64_t r0 = (int64_t)blockIdx.x * TG_MLP_ROWS;
  // phase 1: one thread per row does forward and the scalar output delta
  if (threadIdx.x < TG_MLP_ROWS) {
    const int q = threadIdx.x;
    const int64_t r = r0 + q;
    if (r < nrows) {
      const int64_t src = rows ? rows[r] : r;
      float x[TG_MLP_IN], h1[TG_MLP_H], h2[TG_MLP_H];
      for (int c = 0; c < TG_MLP_IN; ++c) x[c] = (X[src * TG_MLP_IN + c] - stats[c]) / stats[TG_MLP_IN + c];
      const float y = mlp_forward_row(P, x, h1, h2);
      const float err = y - Y[src];
      dys[q] = 2.0f * err / (float)total;
      for (int c = 0; c < TG_MLP_IN; ++c) xs[q][c] = x[c];
      for (int a = 0; a < TG_MLP_H; ++a) { h1s[q][a] = h1[a]; h2s[q][a] = h2[a]; }
    } else {
      dys[q] = 0.0f;
      for (int c = 0; c < TG_MLP_IN; ++c) xs[q][c] = 0.0f;
      for (int a = 0; a < TG_MLP_H; ++a) { h1s[q][a] = 0.0f; h2s[q][a] = 0.0f; }
    }
  }
  __syncthreads();
  // phase 2: deltas, threads over (row, unit)
  for (int z = threadIdx.x; z < TG_MLP_ROWS * TG_MLP_H; z += blockDim.x) {
    const int q = z / TG_MLP_H, a = z % TG_MLP_H;
    d2s[q][a] = h2s[q][a] > 0.0f ? dys[q] * P[TG_MLP_OFF_W3 + a] : 0.0f;
  }
  __syncthreads();
  for (int z = threadIdx.x; z < TG_MLP_ROWS * TG_MLP_H; z += blockDim.x) {
    const int q = z / TG_MLP_H, b = z % TG_MLP_H;
    float s = 0.0f;
    for (int a = 0; a < TG_MLP_H; ++a) s = fmaf(P[TG_MLP_OFF_W2 + a * TG_MLP_H + b], d2s[q][a], s);
    d1s[q][b] = h1s[q][b] > 0.0f ? s : 0.0f;
  }
  __syncthreads();
  // phase 3: parameter gradients summed over the rows in a fixed order
  float* out = partial + (int64_t)blockIdx.x * TG_MLP_NPARAM;
  for (int p = threadIdx.x; p < TG_MLP_NPARAM; p += blockDim.x) {
    float g = 0.0f;
    if (p < TG_MLP_OFF_B1) {
      const int a = p / TG_MLP_IN, c = p % TG_MLP_IN;
      for (int q = 0; q < TG_MLP_ROWS; ++q) g = fmaf(d1s[q][a], xs[q][c], g);
    } else if (p < TG_MLP_OFF_W2) {
      const int a = p - TG_MLP_OFF_B1;
      for (int q = 0; q < TG_MLP_ROWS; ++q) g += d1s[q][a];
    } else if (p < TG_MLP_OFF_B2) {
      const int a = (p - TG_MLP_OFF_W2) / TG_MLP_H, b = (p - TG_MLP_OFF_W2) % TG_MLP_H;
      for (int q = 0; q < TG_MLP_ROWS; ++q) g = fmaf(d2s[q][a], h1s[q][b], g);
    } else if (p < TG_MLP_OFF_W3) {
      const int a = p - TG_MLP_OFF_B2;
      for (int q = 0; q < TG_MLP_ROWS; ++q) g += d2s[q][a];
    } else if (p < TG_MLP_OFF_B3) {
      const int a = p - TG_MLP_OFF_W3;
      for (int q = 0; q < TG_MLP_ROWS; ++q) g = fmaf(dys[q], h2s[q][a], g);
    } else {
      for (int q = 0; q < TG_MLP_ROWS; ++q) g += dys[q];
    }
    out[p] = g;
  }
  if (threadIdx.x == 0) {
    float l = 0.0f;
    for (int q = 0; q < TG_MLP_ROWS; ++q) {
      const float e = dys[q] * (float)total * 0.5f;   // = err
      l = fmaf(e, e, l);
    }
    partial_loss[blockIdx.x] = l / (float)total;
  }
}

// grad[p] = sum over partials in block order; loss likewise.
__global__ void k_mlp_reduce(int nblocks, const float* __restrict__ partial, const float* __restrict__ partial_loss,
                             float* __restrict__ grad, float* __restrict__ loss) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < TG_MLP_NPARAM; p += gridDim.x * blockDim.x) {
    float g = 0.0f;
    for (int b = 0; b < nblocks; ++b) g += partial[(int64_t)b * TG_MLP_NPARAM + p];
    grad[p] = g;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && loss) {
    float l = 0.0f;
    for (int b = 0; b < nblocks; ++b) l += partial_loss[b];
    *loss = l;
  }
}

// Adam on the fp32 master copy, then the bf16 copy used by the kernels.
__global__ void k_mlp_adam(float* __restrict__ W, float* __restrict__ M, float* __restrict__ V,
                           const float* __restrict__ grad, uint16_t* __restrict__ Wbf, float lr, float b1, float b2,
                           float eps, float c1, float c2) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < TG_MLP_NPARAM; p += gridDim.x * blockDim.x) {
    const float g = grad[p];
    const float m = b1 * M[p] + (1.0f - b1) * g;
    const float v = b2 * V[p] + (1.0f - b2) * g * g;
    M[p] = m;
    V[p] = v;
    const float w = W[p] - lr * (m / c1) / (sqrtf(v / c2) + eps);
    W[p] = w;
    uint32_t u;
    const float r = bf16_round(w);
    memcpy(&u, &r, 4);
    Wbf[p] = (uint16_t)(u >> 16);
  }
}

__global__ void k_mlp_to_bf16(const float* __restrict__ W, uint16_t* __restrict__ Wbf) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < TG_MLP_NPARAM; p += gridDim.x * blockDim.x) {
    uint32_t u;
    const float r = bf16_round(W[p]);
    memcpy(&u, &r, 4);
    Wbf[p] = (uint16_t)(u >> 16);
  }
}

__global__ void k_gather_f32(int64_t n, const int32_t* __restrict__ idx, const float* __restrict__ src,
                             float* __restrict__ dst) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
    dst[q] = src[idx[q]];
}

// log2(1 + work) of each sampled edge
__global__ void k_work_to_target(int64_t n, const uint64_t* __restrict__ work, float* __restrict__ Y) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
    Y[q] = (float)log2(1.0 + (double)work[q]);
}

__global__ void k_max_tsum(int64_t count, const int32_t* __restrict__ list, const uint32_t* __restrict__ tau, int L,
                           uint32_t* __restrict__ out) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < count; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = list[q];
    uint32_t t = 0;
    for (int u = 0; u < L; ++u) t += tau[e * L + u];
    atomicMax(out, t);
  }
}

__global__ void k_sample_flags(int64_t m, uint64_t seed, uint64_t thr, int32_t* __restrict__ flag) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
    uint64_t z = seed * 0x9E3779B97F4A7C15ull + (uint64_t)e * 0xD1B54A32D192ED03ull + 0x8CB92BA72F3D8DD7ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    flag[e] = z < thr ? 1 : 0;
  }
}

__global__ void k_compact(int64_t m, const int32_t* __restrict__ flag, const int32_t* __restrict__ pos,
                          int32_t* __restrict__ list) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x)
    if (flag[e]) list[pos[e]] = (int32_t)e;
}

}  // namespace tg
