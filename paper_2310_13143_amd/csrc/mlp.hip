// FP32 multilayer perceptron of the learned ADMM warm start on the gfx950
// matrix cores: forward pass, back-propagation with per-block gradient
// partials, fixed-order reduction, Adam.
//
// A block of 4 waves processes tiles of 64 samples.  Every layer is a
// product (rows x K) . (K x 64 samples) computed with
// v_mfma_f32_16x16x4_f32: wave w owns rows 16w..16w+15 of the hidden
// layers, so the weight operands of a wave stay in registers for all
// tiles.  Activations live in LDS as rows of 64 samples with an odd row
// stride (65).  Within a product of depth K = 4 n, lane group g = lane / 16
// supplies the terms k = n g + j at step j (any order of the k terms gives
// the same sum up to rounding), so the operands read either 2 rows x 16
// samples or 16 rows x 2 samples per 32 lanes, both free of bank conflicts,
// at addresses that are a per-lane base plus a constant.  Weight gradients
// accumulate in MFMA accumulators across the block's tiles and are written
// once per block.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>

#include "acopf_mlp.h"
#include "errors.h"

using namespace acopf;

namespace {

constexpr int H = ACOPF_MLP_HIDDEN;  // hidden width (4 row tiles of 16)
constexpr int TS = 64;               // samples per tile
constexpr int kThreads = 256;        // 4 waves
constexpr int kMaxBlocks = 512;  // two resident blocks per CU (54 KB of LDS each)
constexpr int kMaxIn = 64, kMaxOut = 16;

typedef float f4 __attribute__((ext_vector_type(4)));

// D = A B + C with A 16x4, B 4x16, C, D 16x16.  Lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16] and holds D[4 (l / 16) + r][l % 16] in element r.
__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

constexpr int LD = TS + 1;  // LDS row stride (odd)

struct Offsets {
  int w1, b1, w2, b2, w3, b3, count;
};

__host__ __device__ inline Offsets offsets(int n_in, int n_out) {
  Offsets o;
  o.w1 = 0;
  o.b1 = o.w1 + H * n_in;
  o.w2 = o.b1 + H;
  o.b2 = o.w2 + H * H;
  o.w3 = o.b2 + H;
  o.b3 = o.w3 + n_out * H;
  o.count = o.b3 + n_out;
  return o;
}

inline bool sizes_ok(int n_in, int n_out) { return n_in >= 1 && n_in <= kMaxIn && n_out >= 1 && n_out <= kMaxOut; }

inline int blocks_for_samples(long long n) {
  return (int)std::min<long long>((n + TS - 1) / TS, kMaxBlocks);
}

// kTrain = false: outputs Y.  kTrain = true: loss and gradient partials of
// this block at part[blockIdx.x * (count + 1)] (the loss sum last); dY is
// scaled by inv_scale = 2 / (n n_out).
template <bool kTrain>
__global__ void __launch_bounds__(kThreads) k_mlp(const float* __restrict__ th, int n_in, int n_out,
                                                  const float* __restrict__ X, long long ldx,
                                                  const float* __restrict__ T, long long ldt, long long n,
                                                  float* __restrict__ Y, long long ldy, float* __restrict__ part,
                                                  float inv_scale) {
  __shared__ float sX[kMaxIn * LD];
  __shared__ float sH1[H * LD];
  __shared__ float sH2[H * LD];
  __shared__ float sD[kMaxOut * LD];
  __shared__ float sRed[kThreads / 64];

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const Offsets P = offsets(n_in, n_out);
  const int k1 = (n_in + 3) >> 2;          // steps of layer 1 (depth 4 k1)
  const int nc1 = (n_in + 15) >> 4;        // column tiles of dW1
  const int xrows = 16 * nc1;              // rows of sX kept finite (>= 4 k1)

  // weight operands of this wave (zero outside the network's sizes)
  float a1[16], a2[16], a3[16];
#pragma unroll
  for (int ks = 0; ks < 16; ++ks) {
    const int k = k1 * lk + ks;
    a1[ks] = (ks < k1 && k < n_in) ? th[P.w1 + (16 * wv + li) * n_in + k] : 0.0f;
    a2[ks] = th[P.w2 + (16 * wv + li) * H + 16 * lk + ks];
    a3[ks] = (li < n_out) ? th[P.w3 + li * H + 16 * lk + ks] : 0.0f;
  }
  float bb1[4], bb2[4], bb3[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    bb1[r] = th[P.b1 + 16 * wv + 4 * lk + r];
    bb2[r] = th[P.b2 + 16 * wv + 4 * lk + r];
    bb3[r] = (4 * lk + r < n_out) ? th[P.b3 + 4 * lk + r] : 0.0f;
  }
  float a3t[4], a2t[16];
  f4 gW1[4], gW2[4], gW3;
  float loss = 0.0f;
  float gb1 = 0.0f, gb2 = 0.0f, gb3 = 0.0f;  // bias gradients of row tid (tid < 64, < 16)
  if (kTrain) {
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int o = 4 * lk + ks;
      a3t[ks] = (o < n_out) ? th[P.w3 + o * H + 16 * wv + li] : 0.0f;
    }
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) a2t[ks] = th[P.w2 + (16 * lk + ks) * H + 16 * wv + li];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      gW1[c] = f4{0.0f, 0.0f, 0.0f, 0.0f};
      gW2[c] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    }
    gW3 = f4{0.0f, 0.0f, 0.0f, 0.0f};
  }
  // per-lane bases of the two operand patterns and of the accumulator rows
  const int rowA = (16 * lk) * LD + li;          // row 16 lk + ks, sample 16 c + li: + ks LD + 16 c
  const int rowX = (k1 * lk) * LD + li;          // layer 1: row k1 lk + ks
  const int rowT = (4 * lk) * LD + li;           // depth 16: row 4 lk + ks
  const int colB = li * LD + 16 * lk;            // row 16 t + li, sample 16 lk + ks: + 16 t LD + ks
  const int accw = (16 * wv + 4 * lk) * LD + li; // accumulator element r of column tile c: + r LD + 16 c

  for (long long tile = blockIdx.x; tile * TS < n; tile += gridDim.x) {
    const long long n0 = tile * TS;
    const int nv = (int)std::min<long long>(TS, n - n0);
    // stage the inputs (rows past n_in and samples past n are zero)
    for (int e = tid; e < xrows * TS; e += kThreads) {
      const int f = e / TS, s = e % TS;
      sX[f * LD + s] = (f < n_in && s < nv) ? X[f * ldx + n0 + s] : 0.0f;
    }
    __syncthreads();

    // layer 1: H1 = relu(W1 X + b1)
    {
      f4 acc[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] = f4{0.0f, 0.0f, 0.0f, 0.0f};
      for (int ks = 0; ks < k1; ++ks) {
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] = mfma(a1[ks], sX[rowX + ks * LD + 16 * c], acc[c]);
      }
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r) sH1[accw + r * LD + 16 * c] = fmaxf(acc[c][r] + bb1[r], 0.0f);
    }
    __syncthreads();

    // layer 2: H2 = relu(W2 H1 + b2)
    {
      f4 acc[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int ks = 0; ks < 16; ++ks) {
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] = mfma(a2[ks], sH1[rowA + ks * LD + 16 * c], acc[c]);
      }
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r) sH2[accw + r * LD + 16 * c] = fmaxf(acc[c][r] + bb2[r], 0.0f);
    }
    __syncthreads();

    // layer 3: Y = W3 H2 + b3; wave wv takes samples 16 wv .. 16 wv + 15
    f4 y = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) y = mfma(a3[ks], sH2[rowA + ks * LD + 16 * wv], y);
    const int s = 16 * wv + li;
    if (!kTrain) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int o = 4 * lk + r;
        if (o < n_out && s < nv) Y[o * ldy + n0 + s] = y[r] + bb3[r];
      }
      // No barrier needed before the next tile: its first LDS writes go to
      // sX, last read by layer 1 before the barrier that precedes layer 2.
      continue;
    }

    // dY = 2 (Y - T) / (n n_out), zero for padded outputs and samples
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int o = 4 * lk + r;
      float d = 0.0f;
      if (o < n_out && s < nv) d = y[r] + bb3[r] - T[o * ldt + n0 + s];
      loss += d * d;
      sD[o * LD + s] = d * inv_scale;
    }
    __syncthreads();

    // dW3 += dY H2^T (wave wv: columns 16 wv ..) and dH2 = W3^T dY masked
    // by H2 > 0, stored over H2.  Wave wv reads and writes only rows
    // 16 wv .. of sH2 here, so program order suffices between the two.
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) gW3 = mfma(sD[colB + ks], sH2[colB + 16 * wv * LD + ks], gW3);
    if (tid < kMaxOut) {
      float t = 0.0f;
      for (int c = 0; c < TS; ++c) t += sD[tid * LD + c];
      gb3 += t;
    }
    {
      f4 acc[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] = mfma(a3t[ks], sD[rowT + ks * LD + 16 * c], acc[c]);
      }
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int p = accw + r * LD + 16 * c;
          sH2[p] = (sH2[p] > 0.0f) ? acc[c][r] : 0.0f;
        }
    }
    __syncthreads();  // sH2 holds dZ2 for every row

    // dW2 += dZ2 H1^T; db2 += row sums of dZ2; dH1 = W2^T dZ2 (registers)
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) {
      const float a = sH2[colB + 16 * wv * LD + ks];
#pragma unroll
      for (int c = 0; c < 4; ++c) gW2[c] = mfma(a, sH1[colB + 16 * c * LD + ks], gW2[c]);
    }
    if (tid < H) {
      float t = 0.0f;
      for (int c = 0; c < TS; ++c) t += sH2[tid * LD + c];
      gb2 += t;
    }
    f4 dh1[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) dh1[c] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) {
#pragma unroll
      for (int c = 0; c < 4; ++c) dh1[c] = mfma(a2t[ks], sH2[rowA + ks * LD + 16 * c], dh1[c]);
    }
    __syncthreads();  // every wave is done reading H1
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int p = accw + r * LD + 16 * c;
        sH1[p] = (sH1[p] > 0.0f) ? dh1[c][r] : 0.0f;
      }
    __syncthreads();  // sH1 holds dZ1

    // dW1 += dZ1 X^T; db1 += row sums of dZ1
    for (int c = 0; c < nc1; ++c) {
#pragma unroll
      for (int ks = 0; ks < 16; ++ks) gW1[c] = mfma(sH1[colB + 16 * wv * LD + ks], sX[colB + 16 * c * LD + ks], gW1[c]);
    }
    if (tid < H) {
      float t = 0.0f;
      for (int c = 0; c < TS; ++c) t += sH1[tid * LD + c];
      gb1 += t;
    }
    __syncthreads();  // before the next tile overwrites sX, sH1, sH2, sD
  }
  if (!kTrain) return;

  // block partials in parameter order, loss sum last
  float* out = part + (size_t)blockIdx.x * (P.count + 1);
  for (int c = 0; c < nc1; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int f = 16 * c + li;
      if (f < n_in) out[P.w1 + (16 * wv + 4 * lk + r) * n_in + f] = gW1[c][r];
    }
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) out[P.w2 + (16 * wv + 4 * lk + r) * H + 16 * c + li] = gW2[c][r];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int o = 4 * lk + r;
    if (o < n_out) out[P.w3 + o * H + 16 * wv + li] = gW3[r];
  }
  if (tid < H) {
    out[P.b1 + tid] = gb1;
    out[P.b2 + tid] = gb2;
  }
  if (tid < n_out) out[P.b3 + tid] = gb3;
  // loss: wave sums, then the waves in order
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) loss += __shfl_xor(loss, off, 64);
  if (lane == 0) sRed[wv] = loss;
  __syncthreads();
  if (tid == 0) out[P.count] = sRed[0] + sRed[1] + sRed[2] + sRed[3];
}

// grad[p] = sum over blocks of the partials; loss = sum / (n n_out), in two
// levels with a fixed segmentation (results independent of timing):
// k_mlp_reduce_seg sums kSegs contiguous ranges of blocks per entry (block
// order inside a range), k_mlp_reduce_fin adds the kSegs range sums in
// order.  A block of the first kernel serves 64 entries x 4 ranges.
constexpr int kSegs = 32;

// Device scratch of acopf_mlp_gradient_noalloc: the per-block partials and
// range sums of the largest network (64 inputs, 16 outputs) at the block
// cap, (512 + 32) x 9,361 floats = 20.4 MB per device.  Every GPU that
// runs the library holds its own copy until the process ends.
constexpr int kMaxCount = H * kMaxIn + H + H * H + H + kMaxOut * H + kMaxOut;
constexpr size_t kScratchFloats = (size_t)(kMaxBlocks + kSegs) * (kMaxCount + 1);
__device__ __align__(256) float scratch[kScratchFloats];

__global__ void __launch_bounds__(256) k_mlp_reduce_seg(const float* __restrict__ part, int nblk, int count,
                                                        float* __restrict__ seg_out) {
  const int j = threadIdx.x & 63;
  const int seg = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int p = blockIdx.x * 64 + j;
  if (p > count) return;
  const int b0 = seg * nblk / kSegs, b1 = (seg + 1) * nblk / kSegs;
  float t = 0.0f;
  for (int b = b0; b < b1; ++b) t += part[(size_t)b * (count + 1) + p];
  seg_out[(size_t)seg * (count + 1) + p] = t;
}

__global__ void k_mlp_reduce_fin(const float* __restrict__ seg_in, int count, float inv_count,
                                 float* __restrict__ grad, float* __restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > count) return;
  float t = 0.0f;
  for (int k = 0; k < kSegs; ++k) t += seg_in[(size_t)k * (count + 1) + p];
  if (p < count)
    grad[p] = t;
  else
    *loss = t * inv_count;
}

__global__ void k_adam(float* __restrict__ th, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, long long count, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < count;
       p += (long long)gridDim.x * blockDim.x) {
    const float gp = g[p];
    const float mp = b1 * m[p] + (1.0f - b1) * gp;
    const float vp = b2 * v[p] + (1.0f - b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    th[p] -= lr * (mp * c1) / (sqrtf(vp * c2) + eps);
  }
}

// Mean and standard deviation (population, floored) of each row of a
// feature-major array: one block per row, two passes in FP64, fixed-order
// block sums.
__device__ double block_sum_d(double v, double* lds) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  double t = 0.0;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += lds[k];
  __syncthreads();
  return t;
}

__global__ void k_feature_stats(const float* __restrict__ X, long long ldx, long long n, double floor_std,
                               double* __restrict__ mean, double* __restrict__ stdev) {
  __shared__ double lds[kThreads / 64];
  const float* row = X + blockIdx.x * ldx;
  double s = 0.0;
  for (long long i = threadIdx.x; i < n; i += blockDim.x) s += (double)row[i];
  const double m = block_sum_d(s, lds) / (double)n;
  double q = 0.0;
  for (long long i = threadIdx.x; i < n; i += blockDim.x) {
    const double d = (double)row[i] - m;
    q += d * d;
  }
  const double var = block_sum_d(q, lds) / (double)n;
  if (threadIdx.x == 0) {
    mean[blockIdx.x] = m;
    stdev[blockIdx.x] = fmax(sqrt(var), floor_std);
  }
}

// X <- (X - mean) / std per row, clipped to +-clip if clip > 0.
__global__ void k_standardize(float* __restrict__ X, int rows, long long ldx, long long n,
                              const double* __restrict__ mean, const double* __restrict__ stdev, double clip) {
  const long long total = (long long)rows * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(e / n);
    const long long i = e - (long long)r * n;
    double z = ((double)X[r * ldx + i] - mean[r]) / stdev[r];
    if (clip > 0.0) z = fmin(fmax(z, -clip), clip);
    X[r * ldx + i] = (float)z;
  }
}

// Fold x -> (x - in_mean) / in_std into W1, b1 and y -> out_std y + out_mean
// into W3, b3 (one block).
__global__ void k_fold(float* __restrict__ th, int n_in, int n_out, const double* __restrict__ in_mean,
                       const double* __restrict__ in_std, const double* __restrict__ out_mean,
                       const double* __restrict__ out_std) {
  const Offsets P = offsets(n_in, n_out);
  for (int h = threadIdx.x; h < H; h += blockDim.x) {
    double shift = 0.0;
    for (int f = 0; f < n_in; ++f) {
      const double wv = (double)th[P.w1 + h * n_in + f] / in_std[f];
      th[P.w1 + h * n_in + f] = (float)wv;
      shift += wv * in_mean[f];
    }
    th[P.b1 + h] = (float)((double)th[P.b1 + h] - shift);
  }
  for (int e = threadIdx.x; e < n_out * H; e += blockDim.x) {
    const int o = e / H;
    th[P.w3 + e] = (float)((double)th[P.w3 + e] * out_std[o]);
  }
  for (int o = threadIdx.x; o < n_out; o += blockDim.x)
    th[P.b3 + o] = (float)((double)th[P.b3 + o] * out_std[o] + out_mean[o]);
}

// Launches of the gradient (per-block partials, then the fixed-order
// reduction) with the partials at part.  Every entry of part the reduction
// reads is written by the kernel before it: nothing needs clearing.
acopf_status gradient_launch(const float* theta, int n_in, int n_out, const float* X, int64_t ldx, const float* T,
                             int64_t ldt, int64_t n, float* grad, float* loss, float* part, hipStream_t s) {
  const int nblk = blocks_for_samples(n);
  const int count = offsets(n_in, n_out).count;
  const double denom = (double)n * (double)n_out;
  hipLaunchKernelGGL(k_mlp<true>, dim3(nblk), dim3(kThreads), 0, s, theta, (int)n_in, (int)n_out, X,
                     (long long)ldx, T, (long long)ldt, (long long)n, nullptr, 0LL, part, (float)(2.0 / denom));
  float* seg = part + (size_t)nblk * (count + 1);  // kSegs range sums after the block partials
  hipLaunchKernelGGL(k_mlp_reduce_seg, dim3((count + 1 + 63) / 64, kSegs / 4), dim3(256), 0, s, part, nblk, count,
                     seg);
  hipLaunchKernelGGL(k_mlp_reduce_fin, dim3((count + 1 + 255) / 256), dim3(256), 0, s, seg, count,
                     (float)(1.0 / denom), grad, loss);
  HIP_TRY(hipGetLastError());
  return ACOPF_OK;
}

// Device address of `scratch` on the current device, looked up once per
// device (host code never passes the array's own name to a kernel).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_addr[kMaxDevices] = {};

acopf_status scratch_address(float** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(ACOPF_ERR_UNSUPPORTED, "acopf_mlp_gradient_noalloc: device index above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(ACOPF_ERR_HIP, "acopf_mlp_gradient_noalloc: no device address for the scratch array");
    g_scratch_addr[dev] = static_cast<float*>(p);
  }
  *out = g_scratch_addr[dev];
  return ACOPF_OK;
}

static_assert(kScratchFloats * sizeof(float) == ACOPF_MLP_NOALLOC_SCRATCH_BYTES, "scratch size in the header");

}  // namespace

extern "C" {

size_t acopf_mlp_param_count(int32_t n_in, int32_t n_out) {
  if (!sizes_ok(n_in, n_out)) return 0;
  return (size_t)offsets(n_in, n_out).count;
}

size_t acopf_mlp_scratch_bytes(int32_t n_in, int32_t n_out, int64_t n) {
  if (!sizes_ok(n_in, n_out) || n < 1) return 0;
  return (size_t)(blocks_for_samples(n) + kSegs) * (offsets(n_in, n_out).count + 1) * sizeof(float);
}

acopf_status acopf_mlp_forward(const float* theta, int32_t n_in, int32_t n_out, const float* X, int64_t ldx,
                               int64_t n, float* Y, int64_t ldy, void* stream) {
  if (!sizes_ok(n_in, n_out)) return fail(ACOPF_ERR_INVALID_ARG, "acopf_mlp_forward: n_in must be in [1, 64], n_out in [1, 16]");
  if (!theta || !X || !Y || n < 0 || ldx < n || ldy < n)
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_mlp_forward: null array or leading dimension below n");
  if (n == 0) return ACOPF_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_mlp<false>, dim3(blocks_for_samples(n)), dim3(kThreads), 0, s, theta, (int)n_in,
                     (int)n_out, X, (long long)ldx, nullptr, 0LL, (long long)n, Y, (long long)ldy, nullptr, 0.0f);
  HIP_TRY(hipGetLastError());
  return ACOPF_OK;
}

acopf_status acopf_mlp_gradient(const float* theta, int32_t n_in, int32_t n_out, const float* X, int64_t ldx,
                                const float* T, int64_t ldt, int64_t n, float* grad, float* loss, void* scratch,
                                size_t scratch_bytes, void* stream) {
  if (!sizes_ok(n_in, n_out)) return fail(ACOPF_ERR_INVALID_ARG, "acopf_mlp_gradient: n_in must be in [1, 64], n_out in [1, 16]");
  if (!theta || !X || !T || !grad || !loss || !scratch || n < 1 || ldx < n || ldt < n)
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_mlp_gradient: null array, n < 1 or leading dimension below n");
  if (scratch_bytes < acopf_mlp_scratch_bytes(n_in, n_out, n))
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_mlp_gradient: scratch smaller than acopf_mlp_scratch_bytes");
  return gradient_launch(theta, n_in, n_out, X, ldx, T, ldt, n, grad, loss, static_cast<float*>(scratch),
                         static_cast<hipStream_t>(stream));
}

acopf_status acopf_mlp_gradient_noalloc(const float* theta, int32_t n_in, int32_t n_out, const float* X,
                                        int64_t ldx, const float* T, int64_t ldt, int64_t n, float* grad,
                                        float* loss, void* stream) {
  if (!sizes_ok(n_in, n_out))
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_mlp_gradient_noalloc: n_in must be in [1, 64], n_out in [1, 16]");
  if (!theta || !X || !T || !grad || !loss || n < 1 || ldx < n || ldt < n)
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_mlp_gradient_noalloc: null array, n < 1 or leading dimension below n");
  if (acopf_mlp_scratch_bytes(n_in, n_out, n) > ACOPF_MLP_NOALLOC_SCRATCH_BYTES)
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_mlp_gradient_noalloc: the gradient needs more scratch than the "
                                       "library's static array (ACOPF_MLP_NOALLOC_SCRATCH_BYTES)");
  float* part = nullptr;
  const acopf_status rc = scratch_address(&part);
  if (rc != ACOPF_OK) return rc;
  return gradient_launch(theta, n_in, n_out, X, ldx, T, ldt, n, grad, loss, part,
                         static_cast<hipStream_t>(stream));
}

acopf_status acopf_mlp_adam(float* theta, float* m, float* v, const float* grad, int64_t count, int32_t t,
                            float lr, float beta1, float beta2, float eps, void* stream) {
  if (!theta || !m || !v || !grad || count < 0 || t < 1)
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_mlp_adam: null array, count < 0 or t < 1");
  if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && lr >= 0.0f && eps >= 0.0f))
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_mlp_adam: betas must lie in [0, 1), lr and eps >= 0");
  if (count == 0) return ACOPF_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, t)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, t)));
  const int nb = (int)std::min<long long>((count + 255) / 256, 4096);
  hipLaunchKernelGGL(k_adam, dim3(nb), dim3(256), 0, s, theta, m, v, grad, (long long)count, lr, beta1, beta2,
                     eps, c1, c2);
  HIP_TRY(hipGetLastError());
  return ACOPF_OK;
}

acopf_status acopf_mlp_feature_stats(const float* X, int32_t rows, int64_t ldx, int64_t n, double* mean,
                                    double* stdev, void* stream) {
  if (!X || !mean || !stdev || rows < 1 || n < 1 || ldx < n)
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_mlp_feature_stats: null array, empty input or leading dimension below n");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_feature_stats, dim3(rows), dim3(kThreads), 0, s, X, (long long)ldx, (long long)n,
                     (double)ACOPF_MLP_STD_FLOOR, mean, stdev);
  HIP_TRY(hipGetLastError());
  return ACOPF_OK;
}

acopf_status acopf_mlp_standardize(float* X, int32_t rows, int64_t ldx, int64_t n, const double* mean,
                                   const double* stdev, double clip, void* stream) {
  if (!X || !mean || !stdev || rows < 1 || n < 0 || ldx < n || !(clip >= 0.0))
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_mlp_standardize: bad argument");
  if (n == 0) return ACOPF_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const long long total = (long long)rows * n;
  const int nb = (int)std::min<long long>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(k_standardize, dim3(nb), dim3(256), 0, s, X, (int)rows, (long long)ldx, (long long)n, mean,
                     stdev, clip);
  HIP_TRY(hipGetLastError());
  return ACOPF_OK;
}

acopf_status acopf_mlp_fold(float* theta, int32_t n_in, int32_t n_out, const double* in_mean, const double* in_std,
                            const double* out_mean, const double* out_std, void* stream) {
  if (!sizes_ok(n_in, n_out)) return fail(ACOPF_ERR_INVALID_ARG, "acopf_mlp_fold: n_in must be in [1, 64], n_out in [1, 16]");
  if (!theta || !in_mean || !in_std || !out_mean || !out_std)
    return fail(ACOPF_ERR_INVALID_ARG, "acopf_mlp_fold: null array");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_fold, dim3(1), dim3(kThreads), 0, s, theta, (int)n_in, (int)n_out, in_mean, in_std,
                     out_mean, out_std);
  HIP_TRY(hipGetLastError());
  return ACOPF_OK;
}

}  // extern "C"
