// The per-element warm-start network (n_in -> 128 -> 128 -> n_out, ReLU hidden
// layers) on the GPU: inference, training forward/backward and Adam.
//
// Precision contract: weights, the input and both hidden activations are rounded to
// bfloat16 (round to nearest even) where they enter a matrix product; biases and all
// accumulation are FP32. The forward pass runs the three products on bf16 MFMA
// (v_mfma_f32_32x32x8 bf16, FP32 accumulators): one block of 4 wavefronts takes 64
// samples, the input streamed through LDS in bf16 chunks, each wavefront two 32x32
// output tiles per step, the hidden activations staged in LDS as bf16. The backward pass is FP32 (the roundings are the identity there),
// weight gradients by deterministic split-K reductions.
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"
#include "mfma_bf16.h"

namespace dg {

constexpr int MLP_H = 128;

struct MlpDev {
  int n_in, n_out;
  const uint16_t* W1;   // [H][n_in]  bf16
  const float* b1;
  const uint16_t* W2;   // [H][H]
  const float* b2;
  const uint16_t* W3;   // [n_out][H]
  const float* b3;
};

// Forward of FW_ROWS = 64 samples per block (256 threads, 4 wavefronts). X: fp32
// [n][n_in], rounded to bf16 once per block: it streams through LDS in chunks of FW_KC
// columns (coalesced 16-byte loads, the next chunk's loads in flight while the current
// one is multiplied), so each input byte is read from memory once. Each wavefront holds
// two 32x32 accumulator tiles (the block's two row tiles) per output column tile, so two
// independent MFMA chains alternate. Every product keeps the k order of a single chain
// over k = 0, 8, 16, ... Optional outputs for the backward pass: Z1, H1, Z2, H2 (fp32
// [n][H], the H rounded), Y: fp32 [n][n_out].
constexpr int FW_ROWS = 64, FW_KC = 128, FW_LD = FW_KC + 8, FW_HLD = MLP_H + 8;
constexpr int FW_NLD = 8;   // 16-byte loads per thread per chunk: FW_ROWS * FW_KC / (4 * 256)
static_assert(FW_NLD * 4 * 256 == FW_ROWS * FW_KC, "chunk staging");
static_assert(FW_LD == FW_HLD, "the hidden layers reuse the input buffers");

__device__ inline void fw_load_chunk(const float* __restrict__ X, int64_t m0, int64_t n, int n_in, int k0,
                                     float4 (&v)[FW_NLD]) {
  constexpr int C4 = FW_KC / 4;   // 16-byte loads per row
  const int kc = min(FW_KC, n_in - k0);
  for (int i = 0; i < FW_NLD; ++i) {
    const int q = threadIdx.x + 256 * i, row = q / C4, c = (q % C4) * 4;
    const int64_t m = m0 + row;
    v[i] = (m < n && c < kc) ? *reinterpret_cast<const float4*>(X + m * n_in + k0 + c) : make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

__device__ inline void fw_store_chunk(uint16_t* __restrict__ xs, const float4 (&v)[FW_NLD]) {
  constexpr int C4 = FW_KC / 4;
  for (int i = 0; i < FW_NLD; ++i) {
    const int q = threadIdx.x + 256 * i, row = q / C4, c = (q % C4) * 4;
    const uint32_t lo = (uint32_t)f2bf(v[i].x) | ((uint32_t)f2bf(v[i].y) << 16);
    const uint32_t hi = (uint32_t)f2bf(v[i].z) | ((uint32_t)f2bf(v[i].w) << 16);
    *reinterpret_cast<uint2*>(xs + row * FW_LD + c) = make_uint2(lo, hi);
  }
}

// two row tiles of one 32-column output tile: acc[t] += A(rows 32 t.., K) B^T, A bf16 in LDS
// (row stride a_ld), B bf16 in global memory (row = output column, stride b_ld). The
// fixed-length form is unrolled, so the B fragments of all its k steps are loaded
// before the first product waits for one.
template <int KS>
__device__ inline void fw_tiles_fixed(v16f (&acc)[2], const uint16_t* A, int a_ld, const uint16_t* B, int b_ld) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 31, kq = (lane >> 5) * 4;
  v4s b[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s) b[s] = *reinterpret_cast<const v4s*>(B + r * b_ld + 8 * s + kq);
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const v4s a0 = *reinterpret_cast<const v4s*>(A + r * a_ld + 8 * s + kq);
    const v4s a1 = *reinterpret_cast<const v4s*>(A + (32 + r) * a_ld + 8 * s + kq);
    acc[0] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a0, b[s], acc[0], 0, 0, 0);
    acc[1] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a1, b[s], acc[1], 0, 0, 0);
  }
}

__device__ inline void fw_tiles(v16f (&acc)[2], const uint16_t* A, int a_ld, const uint16_t* B, int b_ld, int K) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 31, kq = (lane >> 5) * 4;
  for (int k0 = 0; k0 < K; k0 += 8) {
    const v4s b = *reinterpret_cast<const v4s*>(B + r * b_ld + k0 + kq);
    const v4s a0 = *reinterpret_cast<const v4s*>(A + r * a_ld + k0 + kq);
    const v4s a1 = *reinterpret_cast<const v4s*>(A + (32 + r) * a_ld + k0 + kq);
    acc[0] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a0, b, acc[0], 0, 0, 0);
    acc[1] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a1, b, acc[1], 0, 0, 0);
  }
}

// bias, ReLU and bf16 rounding of a hidden layer's two tiles (columns 32 w..), into LDS and
// optionally Z / H in global memory
__device__ inline void fw_hidden_out(const v16f (&acc)[2], const float* __restrict__ bias, int wave, int64_t m0,
                                     int64_t n, uint16_t* sh, float* __restrict__ Z, float* __restrict__ Hout) {
  const int lane = threadIdx.x & 63;
  const int j = 32 * wave + (lane & 31);
  for (int t = 0; t < 2; ++t)
    for (int a = 0; a < 16; ++a) {
      const int row = 32 * t + mfma_out_row(a);
      const float z = acc[t][a] + bias[j];
      const uint16_t hb = f2bf(z > 0.f ? z : 0.f);
      sh[row * FW_HLD + j] = hb;
      const int64_t m = m0 + row;
      if (Z && m < n) {
        Z[m * MLP_H + j] = z;
        Hout[m * MLP_H + j] = bf2f(hb);
      }
    }
}

__global__ __launch_bounds__(256) void k_mlp_forward(MlpDev M, int64_t n, const float* __restrict__ X,
                                                     float* __restrict__ Y, float* __restrict__ Z1,
                                                     float* __restrict__ H1, float* __restrict__ Z2,
                                                     float* __restrict__ H2) {
  // two input chunks (bf16) during layer 1; afterwards the same space holds the two
  // hidden layers (bf16): the last chunk loop ends with a barrier
  __shared__ __align__(16) uint16_t xs[2][FW_ROWS * FW_LD];
  uint16_t* sh = xs[0];
  uint16_t* sh2 = xs[1];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t m0 = (int64_t)blockIdx.x * FW_ROWS;
  // ---- layer 1: wave w computes hidden units [32 w, 32 w + 32) of the 64 samples
  {
    const int nch = (M.n_in + FW_KC - 1) / FW_KC;
    const uint16_t* W1w = M.W1 + (size_t)(32 * wave) * M.n_in;
    float4 pre[FW_NLD];
    fw_load_chunk(X, m0, n, M.n_in, 0, pre);
    fw_store_chunk(xs[0], pre);
    __syncthreads();
    v16f acc[2] = {};
    for (int ch = 0; ch < nch; ++ch) {
      const int k0 = ch * FW_KC, kc = min(FW_KC, M.n_in - k0), buf = ch & 1;
      if (ch + 1 < nch) fw_load_chunk(X, m0, n, M.n_in, k0 + FW_KC, pre);
      if (kc == FW_KC)
        fw_tiles_fixed<FW_KC / 8>(acc, xs[buf], FW_LD, W1w + k0, M.n_in);
      else
        fw_tiles(acc, xs[buf], FW_LD, W1w + k0, M.n_in, kc);
      if (ch + 1 < nch) fw_store_chunk(xs[buf ^ 1], pre);
      __syncthreads();
    }
    fw_hidden_out(acc, M.b1, wave, m0, n, sh, Z1, H1);
  }
  __syncthreads();
  // ---- layer 2
  {
    v16f acc[2] = {};
    fw_tiles_fixed<MLP_H / 8>(acc, sh, FW_HLD, M.W2 + (size_t)(32 * wave) * MLP_H, MLP_H);
    fw_hidden_out(acc, M.b2, wave, m0, n, sh2, Z2, H2);
  }
  __syncthreads();
  // ---- layer 3: n_out / 32 column tiles over the 4 waves
  for (int tile = wave; tile < M.n_out / 32; tile += 4) {
    v16f acc[2] = {};
    fw_tiles_fixed<MLP_H / 8>(acc, sh2, FW_HLD, M.W3 + (size_t)(32 * tile) * MLP_H, MLP_H);
    const int j = 32 * tile + (lane & 31);
    for (int t = 0; t < 2; ++t)
      for (int a = 0; a < 16; ++a) {
        const int64_t m = m0 + 32 * t + mfma_out_row(a);
        if (m < n) Y[m * M.n_out + j] = acc[t][a] + M.b3[j];
      }
  }
}

// dY = 2 (Y - T) / (n n_out); per-block partial sums of the squared error
__global__ __launch_bounds__(256) void k_mse_grad(int64_t cnt, float scale, const float* __restrict__ Y,
                                                  const float* __restrict__ T, float* __restrict__ dY,
                                                  double* __restrict__ part) {
  __shared__ double red[256];
  double acc = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x) {
    const float d = Y[i] - T[i];
    dY[i] = 2.0f * d * scale;
    acc += (double)d * (double)d;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// C[m][j] = (sum_k A[m][k] * B[k][j]) * (mask ? (Zm[m][j] > 0) : 1); A fp32 [n][K], B given as
// bf16 weights W[k][j] with row length ldw (B = W: dH = dZ W)
__global__ __launch_bounds__(256) void k_gemm_dgrad(int64_t n, int K, int N, const float* __restrict__ A,
                                                    const uint16_t* __restrict__ W, const float* __restrict__ Zm,
                                                    float* __restrict__ C) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * N) return;
  const int64_t m = idx / N;
  const int j = (int)(idx % N);
  float s = 0.f;
  for (int k = 0; k < K; ++k) s += A[m * K + k] * bf2f(W[(size_t)k * N + j]);
  if (Zm && !(Zm[idx] > 0.f)) s = 0.f;
  C[idx] = s;
}

// split-K weight gradient: part[chunk][p][q] = sum_{m in chunk} A[m][p] * B[m][q]; B may be
// the bf16-rounded network input given in fp32 (rounded here when round_b)
__global__ __launch_bounds__(256) void k_gemm_wgrad(int64_t n, int P, int Q, int64_t chunk, const float* __restrict__ A,
                                                    const float* __restrict__ B, int round_b,
                                                    float* __restrict__ part) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (idx >= (int64_t)P * Q) return;
  const int p = (int)(idx / Q), q = (int)(idx % Q);
  const int64_t m0 = c * chunk, m1 = m0 + chunk < n ? m0 + chunk : n;
  float s = 0.f;
  for (int64_t m = m0; m < m1; ++m) {
    float b = B[m * Q + q];
    if (round_b) b = bf2f(f2bf(b));
    s += A[m * P + p] * b;
  }
  part[(int64_t)c * P * Q + idx] = s;
}

// bias gradient split-K: part[chunk][p] = sum_{m in chunk} A[m][p]
__global__ __launch_bounds__(256) void k_colsum(int64_t n, int P, int64_t chunk, const float* __restrict__ A,
                                                float* __restrict__ part) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (p >= P) return;
  const int64_t m0 = c * chunk, m1 = m0 + chunk < n ? m0 + chunk : n;
  float s = 0.f;
  for (int64_t m = m0; m < m1; ++m) s += A[m * P + p];
  part[(int64_t)c * P + p] = s;
}

__global__ __launch_bounds__(256) void k_sum_chunks(int64_t len, int nchunk, const float* __restrict__ part,
                                                    float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  double s = 0;
  for (int c = 0; c < nchunk; ++c) s += part[(int64_t)c * len + i];
  out[i] = (float)s;
}

// Adam on the fp32 master parameters; refresh of the bf16 weight copies
__global__ __launch_bounds__(256) void k_adam(int64_t len, float lr, float b1, float b2, float eps, float c1, float c2,
                                              const float* __restrict__ g, float* __restrict__ p,
                                              float* __restrict__ m, float* __restrict__ v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// x[r][k] = (x[r][k] - mean[k]) / scale[k]
__global__ void k_affine_rows(int64_t n, int width, const float* __restrict__ mean, const float* __restrict__ scale,
                              float* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * width) return;
  const int k = (int)(i % width);
  x[i] = (x[i] - mean[k]) / scale[k];
}

__global__ void k_to_bf16(int64_t len, const float* __restrict__ x, uint16_t* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) y[i] = f2bf(x[i]);
}

}  // namespace dg

// ------------------------------------------------------------------------- handle
struct dg_mlp_s {
  int n_in = 0, n_out = 0;
  int64_t len = 0;                         // packed parameter count
  int64_t off[7] = {};                     // offsets of W1 b1 W2 b2 W3 b3 in the packed vector
  float* p = nullptr;                      // fp32 master parameters (packed)
  float* g = nullptr;                      // gradients (packed)
  float* m = nullptr;
  float* v = nullptr;
  uint16_t* wb = nullptr;                  // bf16 copies of the packed vector (weights used)
  int64_t adam_t = 0;
  // training scratch
  int64_t cap = 0;
  float *Y = nullptr, *dY = nullptr, *Z1 = nullptr, *H1 = nullptr, *Z2 = nullptr, *H2 = nullptr, *dH = nullptr,
        *dZ = nullptr, *part = nullptr;
  double* dpart = nullptr;
  int64_t part_len = 0;

  dg::MlpDev dev() const {
    return dg::MlpDev{n_in,          n_out, wb + off[0], p + off[1], wb + off[2], p + off[3],
                      wb + off[4], p + off[5]};
  }
};

namespace dg {

int mlp_n_in(const dg_mlp_s* m) { return m->n_in; }
int mlp_n_out(const dg_mlp_s* m) { return m->n_out; }

static void mlp_free_scratch(dg_mlp_s* m) {
  float* ptrs[] = {m->Y, m->dY, m->Z1, m->H1, m->Z2, m->H2, m->dH, m->dZ, m->part};
  for (float* q : ptrs)
    if (q) (void)hipFree(q);
  if (m->dpart) (void)hipFree(m->dpart);
  m->Y = m->dY = m->Z1 = m->H1 = m->Z2 = m->H2 = m->dH = m->dZ = m->part = nullptr;
  m->dpart = nullptr;
  m->cap = 0;
}

static dg_status_t mlp_scratch(dg_mlp_s* m, int64_t n) {
  if (n <= m->cap) return DG_OK;
  mlp_free_scratch(m);
  const int64_t H = MLP_H;
  float** f[] = {&m->Y, &m->dY};
  for (float** q : f)
    if (hipMalloc(q, n * m->n_out * sizeof(float)) != hipSuccess) return DG_ERR_ALLOC;
  float** h[] = {&m->Z1, &m->H1, &m->Z2, &m->H2, &m->dH, &m->dZ};
  for (float** q : h)
    if (hipMalloc(q, n * H * sizeof(float)) != hipSuccess) return DG_ERR_ALLOC;
  m->part_len = 64 * (int64_t)std::max<int64_t>(H * m->n_in, (int64_t)m->n_out * H);
  if (hipMalloc(&m->part, m->part_len * sizeof(float)) != hipSuccess) return DG_ERR_ALLOC;
  if (hipMalloc(&m->dpart, 4096 * sizeof(double)) != hipSuccess) return DG_ERR_ALLOC;
  m->cap = n;
  return DG_OK;
}

dg_status_t mlp_forward(dg_mlp_s* m, const float* X, int64_t n, float* Y, hipStream_t s, bool keep) {
  if (n <= 0) return DG_OK;
  const int blocks = (int)((n + FW_ROWS - 1) / FW_ROWS);
  MlpDev M = m->dev();
  k_mlp_forward<<<blocks, 256, 0, s>>>(M, n, X, Y, keep ? m->Z1 : nullptr, keep ? m->H1 : nullptr,
                                         keep ? m->Z2 : nullptr, keep ? m->H2 : nullptr);
  DG_HIP_CHECK(hipGetLastError());
  return DG_OK;
}

static void wgrad(dg_mlp_s* m, int64_t n, int P, int Q, const float* A, const float* B, int round_b, float* out,
                  hipStream_t s) {
  const int nchunk = (int)std::min<int64_t>(64, (n + 255) / 256);
  const int64_t chunk = (n + nchunk - 1) / nchunk;
  dim3 grid((unsigned)(((int64_t)P * Q + 255) / 256), (unsigned)nchunk);
  k_gemm_wgrad<<<grid, 256, 0, s>>>(n, P, Q, chunk, A, B, round_b, m->part);
  k_sum_chunks<<<(unsigned)(((int64_t)P * Q + 255) / 256), 256, 0, s>>>((int64_t)P * Q, nchunk, m->part, out);
}

static void bgrad(dg_mlp_s* m, int64_t n, int P, const float* A, float* out, hipStream_t s) {
  const int nchunk = (int)std::min<int64_t>(64, (n + 255) / 256);
  const int64_t chunk = (n + nchunk - 1) / nchunk;
  dim3 grid((unsigned)((P + 255) / 256), (unsigned)nchunk);
  k_colsum<<<grid, 256, 0, s>>>(n, P, chunk, A, m->part);
  k_sum_chunks<<<(unsigned)((P + 255) / 256), 256, 0, s>>>(P, nchunk, m->part, out);
}

}  // namespace dg

using namespace dg;

extern "C" {

dg_status_t dg_mlp_create(int32_t n_in, int32_t n_hidden, int32_t n_out, const float* params, dg_mlp_t* out) {
  if (!out || !params || n_in < 8 || n_in % 8 || n_hidden != MLP_H || n_out < 32 || n_out % 32) {
    set_error("dg_mlp_create: needs n_in a multiple of 8, n_hidden = 128, n_out a multiple of 32");
    return DG_ERR_ARG;
  }
  dg_mlp_s* m = new (std::nothrow) dg_mlp_s();
  if (!m) return DG_ERR_ALLOC;
  m->n_in = n_in;
  m->n_out = n_out;
  const int64_t H = MLP_H;
  const int64_t sizes[6] = {H * n_in, H, H * H, H, (int64_t)n_out * H, n_out};
  m->off[0] = 0;
  for (int i = 0; i < 6; ++i) m->off[i + 1] = m->off[i] + sizes[i];
  m->len = m->off[6];
  if (hipMalloc(&m->p, m->len * sizeof(float)) != hipSuccess || hipMalloc(&m->g, m->len * sizeof(float)) != hipSuccess ||
      hipMalloc(&m->m, m->len * sizeof(float)) != hipSuccess || hipMalloc(&m->v, m->len * sizeof(float)) != hipSuccess ||
      hipMalloc(&m->wb, m->len * sizeof(uint16_t)) != hipSuccess) {
    set_error("dg_mlp_create: allocation failed");
    return DG_ERR_ALLOC;
  }
  DG_HIP_CHECK(hipMemcpy(m->p, params, m->len * sizeof(float), hipMemcpyHostToDevice));
  DG_HIP_CHECK(hipMemset(m->m, 0, m->len * sizeof(float)));
  DG_HIP_CHECK(hipMemset(m->v, 0, m->len * sizeof(float)));
  DG_HIP_CHECK(hipMemset(m->g, 0, m->len * sizeof(float)));
  k_to_bf16<<<(unsigned)((m->len + 255) / 256), 256>>>(m->len, m->p, m->wb);
  DG_HIP_CHECK(hipDeviceSynchronize());
  *out = m;
  return DG_OK;
}

dg_status_t dg_mlp_destroy(dg_mlp_t m) {
  if (!m) return DG_OK;
  (void)hipDeviceSynchronize();
  mlp_free_scratch(m);
  void* ptrs[] = {m->p, m->g, m->m, m->v, m->wb};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  delete m;
  return DG_OK;
}

dg_status_t dg_mlp_get_params(dg_mlp_t m, float* params, int64_t len) {
  if (!m || !params || len != m->len) {
    set_error("dg_mlp_get_params: invalid argument");
    return DG_ERR_ARG;
  }
  DG_HIP_CHECK(hipDeviceSynchronize());
  DG_HIP_CHECK(hipMemcpy(params, m->p, m->len * sizeof(float), hipMemcpyDeviceToHost));
  return DG_OK;
}

dg_status_t dg_mlp_forward(dg_mlp_t m, const float* x, int64_t n, float* y, void* stream) {
  if (!m || !x || !y || n < 0 || (reinterpret_cast<uintptr_t>(x) & 15)) {
    set_error("dg_mlp_forward: invalid argument (x must be 16-byte aligned)");
    return DG_ERR_ARG;
  }
  return mlp_forward(m, x, n, y, (hipStream_t)stream, false);
}

dg_status_t dg_mlp_grad(dg_mlp_t m, const float* x, const float* t, int64_t n, double* loss, float* grad_host,
                        void* stream) {
  if (!m || !x || !t || n < 1 || (reinterpret_cast<uintptr_t>(x) & 15)) {
    set_error("dg_mlp_grad: invalid argument (x must be 16-byte aligned)");
    return DG_ERR_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  if (mlp_scratch(m, n) != DG_OK) {
    set_error("dg_mlp_grad: scratch allocation failed");
    return DG_ERR_ALLOC;
  }
  const int H = MLP_H;
  dg_status_t st = mlp_forward(m, x, n, m->Y, s, true);
  if (st != DG_OK) return st;
  const int64_t cnt = n * m->n_out;
  const int nb = (int)std::min<int64_t>(1024, (cnt + 255) / 256);
  k_mse_grad<<<nb, 256, 0, s>>>(cnt, 1.0f / (float)cnt, m->Y, t, m->dY, m->dpart);
  // layer 3
  wgrad(m, n, m->n_out, H, m->dY, m->H2, 0, m->g + m->off[4], s);
  bgrad(m, n, m->n_out, m->dY, m->g + m->off[5], s);
  // dZ2 = (dY W3) * (Z2 > 0)
  k_gemm_dgrad<<<(unsigned)((n * H + 255) / 256), 256, 0, s>>>(n, m->n_out, H, m->dY, m->wb + m->off[4], m->Z2, m->dZ);
  wgrad(m, n, H, H, m->dZ, m->H1, 0, m->g + m->off[2], s);
  bgrad(m, n, H, m->dZ, m->g + m->off[3], s);
  // dZ1 = (dZ2 W2) * (Z1 > 0)
  k_gemm_dgrad<<<(unsigned)((n * H + 255) / 256), 256, 0, s>>>(n, H, H, m->dZ, m->wb + m->off[2], m->Z1, m->dH);
  wgrad(m, n, H, m->n_in, m->dH, x, 1, m->g + m->off[0], s);
  bgrad(m, n, H, m->dH, m->g + m->off[1], s);
  DG_HIP_CHECK(hipGetLastError());
  if (loss) {
    std::vector<double> part(nb);
    DG_HIP_CHECK(hipMemcpyAsync(part.data(), m->dpart, nb * sizeof(double), hipMemcpyDeviceToHost, s));
    DG_HIP_CHECK(hipStreamSynchronize(s));
    double acc = 0;
    for (double v : part) acc += v;
    *loss = acc / (double)cnt;
  }
  if (grad_host) {
    DG_HIP_CHECK(hipStreamSynchronize(s));
    DG_HIP_CHECK(hipMemcpy(grad_host, m->g, m->len * sizeof(float), hipMemcpyDeviceToHost));
  }
  return DG_OK;
}

dg_status_t dg_mlp_adam_step(dg_mlp_t m, float lr, float b1, float b2, float eps, void* stream) {
  if (!m || !(lr > 0)) {
    set_error("dg_mlp_adam_step: invalid argument");
    return DG_ERR_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  m->adam_t += 1;
  const float c1 = 1.f - std::pow(b1, (float)m->adam_t), c2 = 1.f - std::pow(b2, (float)m->adam_t);
  const unsigned blocks = (unsigned)((m->len + 255) / 256);
  k_adam<<<blocks, 256, 0, s>>>(m->len, lr, b1, b2, eps, c1, c2, m->g, m->p, m->m, m->v);
  k_to_bf16<<<blocks, 256, 0, s>>>(m->len, m->p, m->wb);
  DG_HIP_CHECK(hipGetLastError());
  return DG_OK;
}

int64_t dg_mlp_param_count(dg_mlp_t m) { return m ? m->len : 0; }

dg_status_t dg_affine_rows(float* x, int64_t n, int32_t width, const float* mean, const float* scale, void* stream) {
  if (!x || n < 0 || width < 1 || !mean || !scale) {
    set_error("dg_affine_rows: invalid argument");
    return DG_ERR_ARG;
  }
  if (n == 0) return DG_OK;
  hipStream_t s = (hipStream_t)stream;
  k_affine_rows<<<(unsigned)((n * width + 255) / 256), 256, 0, s>>>(n, width, mean, scale, x);
  DG_HIP_CHECK(hipGetLastError());
  return DG_OK;
}

dg_status_t dg_warmstart_set(dg_mesh_t mesh, dg_mlp_t mlp, const float* xm, const float* xs, const float* ym,
                             const float* ys) {
  if (!mesh || mesh->kind != DG_MESH_SHELL) {
    set_error("dg_warmstart_set: needs a shell mesh");
    return DG_ERR_ARG;
  }
  if (!mlp) {
    mesh->ws_mlp = nullptr;
    return DG_OK;
  }
  const int64_t nin = 15 * (int64_t)mesh->N, nout = 5 * (int64_t)mesh->N;
  if (mlp->n_in != nin || mlp->n_out != nout || !xm || !xs || !ym || !ys) {
    set_error("dg_warmstart_set: the network must map 15 N features to 5 N outputs (N nodes per element)");
    return DG_ERR_ARG;
  }
  if (!mesh->ws_norm) DG_HIP_CHECK(hipMalloc(&mesh->ws_norm, (2 * nin + 2 * nout) * sizeof(float)));
  DG_HIP_CHECK(hipMemcpy(mesh->ws_norm, xm, nin * sizeof(float), hipMemcpyHostToDevice));
  DG_HIP_CHECK(hipMemcpy(mesh->ws_norm + nin, xs, nin * sizeof(float), hipMemcpyHostToDevice));
  DG_HIP_CHECK(hipMemcpy(mesh->ws_norm + 2 * nin, ym, nout * sizeof(float), hipMemcpyHostToDevice));
  DG_HIP_CHECK(hipMemcpy(mesh->ws_norm + 2 * nin + nout, ys, nout * sizeof(float), hipMemcpyHostToDevice));
  if (!mesh->ws_X) {
    DG_HIP_CHECK(hipMalloc(&mesh->ws_X, mesh->n_elem * nin * sizeof(float)));
    DG_HIP_CHECK(hipMalloc(&mesh->ws_Y, mesh->n_elem * nout * sizeof(float)));
  }
  mesh->ws_mlp = mlp;
  return DG_OK;
}

dg_status_t dg_warmstart_record(dg_mesh_t mesh, float* x, float* y, int64_t capacity, int32_t every) {
  if (!mesh || mesh->kind != DG_MESH_SHELL || capacity < 0 || (capacity > 0 && (!x || !y || every < 1))) {
    set_error("dg_warmstart_record: invalid argument (needs a shell mesh)");
    return DG_ERR_ARG;
  }
  mesh->rec_x = capacity > 0 ? x : nullptr;
  mesh->rec_y = capacity > 0 ? y : nullptr;
  mesh->rec_cap = capacity;
  mesh->rec_count = 0;
  mesh->rec_every = every > 0 ? every : 1;
  mesh->rec_phase = 0;
  return DG_OK;
}

dg_status_t dg_warmstart_recorded(dg_mesh_t mesh, int64_t* count) {
  if (!mesh || !count) {
    set_error("dg_warmstart_recorded: invalid argument");
    return DG_ERR_ARG;
  }
  *count = mesh->rec_count;
  return DG_OK;
}

}  // extern "C"
