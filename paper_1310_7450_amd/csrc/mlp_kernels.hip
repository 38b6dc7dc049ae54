// lbml: the warm-start network (include/lbml.h) on the gfx950 matrix cores.
//
// Every GEMM is C = A Bt^T with A[m][k] and Bt[n][k] stored as BF16, K
// contiguous, and FP32 accumulation on v_mfma_f32_16x16x32_bf16. The BF16
// operands are formed once, by the kernel that produces them: the input
// conversion, the epilogues of the forward and backward GEMMs (which write
// each activation or gradient both as [row][col] and transposed), and the
// Adam step (which refreshes the weights both as W[out][in] and W^T). Each
// operand buffer is padded with zeros to multiples of 32 in both dimensions,
// so every tile reads whole 16-byte fragments and K needs no tail. One
// wavefront computes a 32 x 32 tile of C as 2 x 2 MFMA blocks: a lane loads
// rows (l % 16) and (l % 16) + 16 of A and of Bt at k = 8 (l / 16) + 0..7
// (one 16-byte load each) per step of 32 in K, with the next step's
// fragments in flight; each fragment feeds two MFMAs. The products are a few
// hundred rows and columns wide: the operands sit in L2, and the kernels are
// bound by latency, so the tile keeps many wavefronts busy instead of staging
// through LDS.
#include "lbml.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short bf16_t;
constexpr int kPad = 32;  // operand padding (rows and columns)
constexpr int kMaxLayers = 16;

// FP32 -> BF16 with round to nearest even (NaN kept quiet).
__host__ __device__ inline bf16_t to_bf16(float f) {
  unsigned int u;
  memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (bf16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}

__device__ inline float sigmoid(float z) { return 1.0f / (1.0f + expf(-z)); }

enum Epilogue { EPI_OUT = 0, EPI_HIDDEN = 1, EPI_DW = 2, EPI_DX = 3 };

struct GemmArgs {
  const bf16_t *A;  // A[m][k], row stride lda (elements)
  const bf16_t *B;  // Bt[n][k], row stride ldb
  int lda, ldb;
  int M, N, K;      // K a multiple of 32; A has roundup(M, 32) rows, Bt roundup(N, 32)
  int tiles_n;
  float *C;         // FP32 result C[m][n] (m < M, n < N), row stride ldc
  int ldc;
  const float *bias;  // EPI_OUT, EPI_HIDDEN: + bias[n]
  float *Z;           // EPI_HIDDEN: pre-activation [m][n] (stride ldc)
  const float *Zp;    // EPI_DX: times SiLU'(Zp[m][n]) (stride ldc)
  bf16_t *Hb;         // EPI_HIDDEN, EPI_DX: BF16 copy [m][n], row stride ldh, zero for n in [N, roundup(N, 32))
  bf16_t *Ht;         // ... and transposed [n][m], row stride ldt, zero for m in [M, roundup(M, 32))
  int ldh, ldt;
};

template <int EPI>
__global__ void __launch_bounds__(64) gemm_kernel(GemmArgs g) {
  const int l = threadIdx.x, r = l & 15, kg = 8 * (l >> 4);
  const int tm = blockIdx.x / g.tiles_n, tn = blockIdx.x % g.tiles_n;
  const int m0 = tm * 32, n0 = tn * 32;
  const bf16_t *a0 = g.A + (long long)(m0 + r) * g.lda + kg, *a1 = a0 + 16LL * g.lda;
  const bf16_t *b0 = g.B + (long long)(n0 + r) * g.ldb + kg, *b1 = b0 + 16LL * g.ldb;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  auto ld = [](const bf16_t *p) __attribute__((always_inline)) { return *reinterpret_cast<const bf16x8 *>(p); };
  bf16x8 fa0 = ld(a0), fa1 = ld(a1), fb0 = ld(b0), fb1 = ld(b1);
  for (int k0 = 0; k0 < g.K; k0 += 32) {
    bf16x8 na0 = fa0, na1 = fa1, nb0 = fb0, nb1 = fb1;
    if (k0 + 32 < g.K) {  // the next step's fragments, in flight during these MFMAs
      na0 = ld(a0 + k0 + 32);
      na1 = ld(a1 + k0 + 32);
      nb0 = ld(b0 + k0 + 32);
      nb1 = ld(b1 + k0 + 32);
    }
    acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa0, fb0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa0, fb1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa1, fb0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa1, fb1, acc[1][1], 0, 0, 0);
    fa0 = na0;
    fa1 = na1;
    fb0 = nb0;
    fb1 = nb1;
  }
  // lane l holds rows 4 (l / 16) + 0..3 of column l % 16 of each 16 x 16 block
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + 16 * i + 4 * (l >> 4) + q, n = n0 + 16 * j + r;
        const bool in = m < g.M && n < g.N;
        float v = acc[i][j][q];
        if (EPI == EPI_OUT || EPI == EPI_HIDDEN) v += in ? g.bias[n] : 0.f;
        if (EPI == EPI_HIDDEN) {
          if (in) g.Z[(long long)m * g.ldc + n] = v;
          v = v * sigmoid(v);
        }
        if (EPI == EPI_DX) {
          if (in) {
            const float z = g.Zp[(long long)m * g.ldc + n], s = sigmoid(z);
            v *= s * (1.0f + z * (1.0f - s));
          }
        }
        if (EPI != EPI_HIDDEN && in) g.C[(long long)m * g.ldc + n] = v;
        if (EPI == EPI_HIDDEN || EPI == EPI_DX) {
          // BF16 operand copies of this result, zero outside [M) x [N)
          const bf16_t b = in ? to_bf16(v) : (bf16_t)0;
          if (m < g.M) g.Hb[(long long)m * g.ldh + n] = b;  // columns up to roundup(N, 32)
          if (n < g.N) g.Ht[(long long)n * g.ldt + m] = b;  // rows m up to roundup(M, 32)
        }
      }
}

// FP32 [rows][cols] -> BF16 [roundup(rows)][roundup(cols)] (ld = padded
// cols) and its transpose [roundup(cols)][roundup(rows)], zero-padded. With
// idx, row r of the result is row idx[r] of x (a gathered minibatch).
__global__ void to_operands_kernel(const float *x, const int32_t *idx, int rows, int cols, bf16_t *xb, int ldb,
                                   bf16_t *xt, int ldt) {
  const int rp = (rows + kPad - 1) / kPad * kPad, cp = (cols + kPad - 1) / kPad * kPad;
  const long long n = (long long)rp * cp;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int rr = (int)(i / cp), cc = (int)(i - (long long)rr * cp);
    const long long src = idx && rr < rows ? (long long)idx[rr] : (long long)rr;
    const bf16_t b = (rr < rows && cc < cols) ? to_bf16(x[src * cols + cc]) : (bf16_t)0;
    xb[(long long)rr * ldb + cc] = b;
    xt[(long long)cc * ldt + rr] = b;
  }
}

// db[n] = sum_m dZ[m][n]: 64 columns per workgroup of 1024 threads, sixteen
// partial sums per column (rows q, q + 16, ... in a fixed order), then a
// fixed tree in LDS, so the result does not depend on scheduling.
__global__ void __launch_bounds__(1024) bias_grad_kernel(const float *dZ, int M, int N, float *db) {
  __shared__ float part[16][64];
  const int c = threadIdx.x & 63, q = threadIdx.x >> 6, n = blockIdx.x * 64 + c;
  float s = 0.f;
  if (n < N) {
#pragma unroll 8
    for (int m = q; m < M; m += 16) s += dZ[(long long)m * N + n];
  }
  part[q][c] = s;
  __syncthreads();
  for (int w = 8; w > 0; w >>= 1) {
    if (q < w) part[q][c] += part[q + w][c];
    __syncthreads();
  }
  if (q == 0 && n < N) db[n] = part[0][c];
}

// dy = 2 (y - t) / count over many workgroups; with loss, per-workgroup
// partial sums of (y - t)^2 into part[blockIdx.x].
__global__ void __launch_bounds__(256) mse_kernel(const float *y, const float *t, const int32_t *idx, int cols,
                                                  long long count, float *dy, double *part) {
  __shared__ double red[256];
  double s = 0.0;
  const float scale = 2.0f / (float)count;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < count; i += 256LL * gridDim.x) {
    // with idx, the target of row r is row idx[r] of t
    const long long r = i / cols, ti = idx ? (long long)idx[r] * cols + (i - r * cols) : i;
    const float d = y[i] - t[ti];
    dy[i] = scale * d;
    s += (double)d * d;
  }
  if (!part) return;
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}
__global__ void __launch_bounds__(64) sum_kernel(const double *part, int n, double scale, double *out) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 64) s += part[i];
  for (int m = 32; m > 0; m >>= 1) s += __shfl_xor(s, m, 64);
  if (threadIdx.x == 0) *out = s * scale;
}

// The weights' BF16 operands of every layer: W[out][in] and W^T, padded.
struct WeightMap {
  int nl;
  long long woff[kMaxLayers];        // offset of W_l in the flat parameters
  long long boff[kMaxLayers];        // offset of b_l (the end of W_l)
  int din[kMaxLayers], dout[kMaxLayers];
  long long wb[kMaxLayers], wt[kMaxLayers];  // element offsets of the BF16 copies
};

__device__ inline void store_weight(const WeightMap &w, bf16_t *pb, long long i, float v) {
  for (int l = 0; l < w.nl; ++l) {
    if (i < w.woff[l] || i >= w.boff[l]) continue;
    const long long j = i - w.woff[l];
    const int o = (int)(j / w.din[l]), in = (int)(j - (long long)o * w.din[l]);
    const int pin = (w.din[l] + kPad - 1) / kPad * kPad, pout = (w.dout[l] + kPad - 1) / kPad * kPad;
    const bf16_t b = to_bf16(v);
    pb[w.wb[l] + (long long)o * pin + in] = b;
    pb[w.wt[l] + (long long)in * pout + o] = b;
  }
}

__global__ void adam_kernel(float *p, const float *g, float *m, float *v, bf16_t *pb, WeightMap w, long long n,
                            float lr, float b1, float b2, float eps, float c1, float c2) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wv = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = wv;
  store_weight(w, pb, i, wv);
}

__global__ void refresh_kernel(const float *p, bf16_t *pb, WeightMap w, long long n) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n) store_weight(w, pb, i, p[i]);
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
int padded(int v) { return (v + kPad - 1) / kPad * kPad; }

struct Plan {
  std::vector<int> dims;
  std::vector<size_t> woff, boff;  // parameter offsets (floats)
  size_t params = 0, max_width = 0;
  int bp = 0, max_pw = 0;          // padded batch and widest padded layer
  WeightMap wm{};
  size_t bf16_weights = 0;          // elements of the padded BF16 weight copies
  size_t off_p = 0, off_g = 0, off_m = 0, off_v = 0, off_pb = 0, off_loss = 0, off_part = 0;
  size_t off_dz[2] = {0, 0};        // FP32 dZ [batch][width]
  size_t off_db[2] = {0, 0}, off_dt[2] = {0, 0};  // BF16 dZ [bp][pw] and dZ^T [pw][bp]
  size_t off_xb = 0, off_xt = 0;    // BF16 input and its transpose
  size_t off_y = 0, off_dy = 0;     // lbml_train_step: output and its gradient
  std::vector<size_t> off_z, off_hb, off_ht;  // per hidden layer: FP32 Z, BF16 H and H^T
  size_t bytes = 0;
};
constexpr int kMsePart = 64;  // workgroups of the loss reduction

bool make_plan(int nl, const int32_t *dims, int max_batch, Plan &P) {
  if (nl < 1 || nl > kMaxLayers || !dims || max_batch < 1) return false;
  P.dims.assign(dims, dims + nl + 1);
  for (int d : P.dims)
    if (d < 1 || d > 65536) return false;
  size_t o = 0;
  for (int l = 0; l < nl; ++l) {
    P.woff.push_back(o);
    o += (size_t)P.dims[l] * P.dims[l + 1];
    P.boff.push_back(o);
    o += P.dims[l + 1];
  }
  P.params = o;
  for (int d : P.dims) {
    P.max_width = std::max(P.max_width, (size_t)d);
    P.max_pw = std::max(P.max_pw, padded(d));
  }
  P.bp = padded(max_batch);
  P.wm.nl = nl;
  size_t e = 0;
  for (int l = 0; l < nl; ++l) {
    P.wm.woff[l] = (long long)P.woff[l];
    P.wm.boff[l] = (long long)P.boff[l];
    P.wm.din[l] = P.dims[l];
    P.wm.dout[l] = P.dims[l + 1];
    P.wm.wb[l] = (long long)e;
    e += (size_t)padded(P.dims[l + 1]) * padded(P.dims[l]);
    P.wm.wt[l] = (long long)e;
    e += (size_t)padded(P.dims[l]) * padded(P.dims[l + 1]);
  }
  P.bf16_weights = e;
  size_t at = 0;
  auto take = [&](size_t b) {
    size_t p = at;
    at = align_up(at + b, 256);
    return p;
  };
  P.off_p = take(4 * P.params);
  P.off_g = take(4 * P.params);
  P.off_m = take(4 * P.params);
  P.off_v = take(4 * P.params);
  P.off_pb = take(2 * P.bf16_weights);
  P.off_loss = take(8);
  P.off_part = take(8 * kMsePart);
  const size_t opnd = 2 * (size_t)P.bp * P.max_pw;
  for (int i = 0; i < 2; ++i) {
    P.off_dz[i] = take(4 * (size_t)max_batch * P.max_width);
    P.off_db[i] = take(opnd);
    P.off_dt[i] = take(opnd);
  }
  P.off_y = take(4 * (size_t)max_batch * P.dims[nl]);
  P.off_dy = take(4 * (size_t)max_batch * P.dims[nl]);
  P.off_xb = take(2 * (size_t)P.bp * padded(P.dims[0]));
  P.off_xt = take(2 * (size_t)P.bp * padded(P.dims[0]));
  for (int l = 0; l < nl; ++l) {
    P.off_z.push_back(take(4 * (size_t)max_batch * P.dims[l + 1]));
    P.off_hb.push_back(take(2 * (size_t)P.bp * padded(P.dims[l + 1])));
    P.off_ht.push_back(take(2 * (size_t)P.bp * padded(P.dims[l + 1])));
  }
  P.bytes = at;
  return true;
}

}  // namespace

struct lbml_net {
  Plan P;
  int nl = 0, max_batch = 0;
  char *ws = nullptr;
  hipStream_t stream = nullptr;
  int last_batch = 0;
  std::string err;
  float *f(size_t off) { return reinterpret_cast<float *>(ws + off); }
  bf16_t *b(size_t off) { return reinterpret_cast<bf16_t *>(ws + off); }
  bf16_t *pb() { return b(P.off_pb); }
};

namespace {

lbml_status fail(lbml_net *h, lbml_status s, const std::string &m) {
  if (h) h->err = m;
  return s;
}

#define MLCHECK(h, call)                                                              \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) return fail((h), -3, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <int EPI>
hipError_t gemm(hipStream_t s, GemmArgs g) {
  g.tiles_n = (g.N + 31) / 32;
  const int tiles = ((g.M + 31) / 32) * g.tiles_n;
  hipLaunchKernelGGL((gemm_kernel<EPI>), dim3(tiles), dim3(64), 0, s, g);
  return hipGetLastError();
}

hipError_t to_operands(hipStream_t s, const float *x, const int32_t *idx, int rows, int cols, bf16_t *xb, int ldb,
                       bf16_t *xt, int ldt) {
  const long long n = (long long)padded(rows) * padded(cols);
  const int blocks = (int)std::min<long long>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(to_operands_kernel, dim3(blocks), dim3(256), 0, s, x, idx, rows, cols, xb, ldb, xt, ldt);
  return hipGetLastError();
}

}  // namespace

extern "C" {

lbml_status lbml_workspace_bytes(int32_t nl, const int32_t *dims, int32_t max_batch, size_t *bytes) {
  Plan P;
  if (!bytes || !make_plan(nl, dims, max_batch, P)) return -1;
  *bytes = P.bytes;
  return 0;
}

lbml_status lbml_param_count(int32_t nl, const int32_t *dims, size_t *count) {
  Plan P;
  if (!count || !make_plan(nl, dims, 1, P)) return -1;
  *count = P.params;
  return 0;
}

lbml_status lbml_create(int32_t nl, const int32_t *dims, int32_t max_batch, void *ws, size_t ws_bytes,
                        void *stream, lbml_net **out) {
  if (!out) return -1;
  *out = nullptr;
  Plan P;
  if (!make_plan(nl, dims, max_batch, P)) return -1;
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255)) return -1;
  if (ws_bytes < P.bytes) return -2;
  lbml_net *h = new (std::nothrow) lbml_net();
  if (!h) return -2;
  h->P = P;
  h->nl = nl;
  h->max_batch = max_batch;
  h->ws = static_cast<char *>(ws);
  h->stream = static_cast<hipStream_t>(stream);  // NULL: the default stream
  // zero everything: parameters, gradients, moments, and the padding of the
  // BF16 operands, which no kernel writes (outside any graph)
  if (hipMemsetAsync(h->ws, 0, P.bytes, h->stream) != hipSuccess || hipStreamSynchronize(h->stream) != hipSuccess) {
    lbml_destroy(h);
    return -3;
  }
  *out = h;
  return 0;
}

lbml_status lbml_destroy(lbml_net *h) {
  if (!h) return 0;
  (void)hipStreamSynchronize(h->stream);
  delete h;
  return 0;
}

lbml_status lbml_set_params(lbml_net *h, const float *p, size_t n) {
  if (!h) return -1;
  if (!p || n != h->P.params) return fail(h, -1, "parameter count mismatch");
  MLCHECK(h, hipMemcpyAsync(h->f(h->P.off_p), p, 4 * n, hipMemcpyHostToDevice, h->stream));
  hipLaunchKernelGGL(refresh_kernel, dim3((n + 255) / 256), dim3(256), 0, h->stream, h->f(h->P.off_p), h->pb(),
                     h->P.wm, (long long)n);
  MLCHECK(h, hipGetLastError());
  MLCHECK(h, hipStreamSynchronize(h->stream));
  return 0;
}

lbml_status lbml_get_params(lbml_net *h, float *p, size_t n) {
  if (!h) return -1;
  if (!p || n != h->P.params) return fail(h, -1, "parameter count mismatch");
  MLCHECK(h, hipMemcpyAsync(p, h->f(h->P.off_p), 4 * n, hipMemcpyDeviceToHost, h->stream));
  MLCHECK(h, hipStreamSynchronize(h->stream));
  return 0;
}

lbml_status lbml_get_grads(lbml_net *h, float *g, size_t n) {
  if (!h) return -1;
  if (!g || n != h->P.params) return fail(h, -1, "parameter count mismatch");
  MLCHECK(h, hipMemcpyAsync(g, h->f(h->P.off_g), 4 * n, hipMemcpyDeviceToHost, h->stream));
  MLCHECK(h, hipStreamSynchronize(h->stream));
  return 0;
}

}  // extern "C"

namespace {

lbml_status forward_impl(lbml_net *h, const float *x, const int32_t *idx, int32_t batch, float *y) {
  const Plan &P = h->P;
  // the input as BF16 operands: [batch][in] for this GEMM, transposed for dW
  MLCHECK(h, to_operands(h->stream, x, idx, batch, P.dims[0], h->b(P.off_xb), padded(P.dims[0]), h->b(P.off_xt),
                         P.bp));
  const bf16_t *in = h->b(P.off_xb);
  for (int l = 0; l < h->nl; ++l) {
    const int din = P.dims[l], dout = P.dims[l + 1];
    GemmArgs g{};
    g.A = in;
    g.lda = padded(din);
    g.B = h->pb() + P.wm.wb[l];  // W[out][in]: row n = out, K = in
    g.ldb = padded(din);
    g.M = batch;
    g.N = dout;
    g.K = padded(din);
    g.ldc = dout;
    g.bias = h->f(P.off_p) + P.boff[l];
    if (l == h->nl - 1) {
      g.C = y;
      MLCHECK(h, gemm<EPI_OUT>(h->stream, g));
    } else {
      g.Z = h->f(P.off_z[l]);
      g.Hb = h->b(P.off_hb[l]);
      g.ldh = padded(dout);
      g.Ht = h->b(P.off_ht[l]);
      g.ldt = P.bp;
      MLCHECK(h, gemm<EPI_HIDDEN>(h->stream, g));
      in = g.Hb;
    }
  }
  h->last_batch = batch;
  return 0;
}

lbml_status mse_impl(lbml_net *h, const float *y, const float *t, const int32_t *idx, int32_t batch, float *dy,
                     double *host_loss) {
  const int cols = h->P.dims[h->nl];
  const long long count = (long long)batch * cols;
  const int blocks = (int)std::min<long long>((count + 255) / 256, kMsePart);
  double *part = host_loss ? reinterpret_cast<double *>(h->ws + h->P.off_part) : nullptr;
  hipLaunchKernelGGL(mse_kernel, dim3(blocks), dim3(256), 0, h->stream, y, t, idx, cols, count, dy, part);
  MLCHECK(h, hipGetLastError());
  if (host_loss) {
    double *dl = reinterpret_cast<double *>(h->ws + h->P.off_loss);
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(64), 0, h->stream, part, blocks, 1.0 / (double)count, dl);
    MLCHECK(h, hipGetLastError());
    MLCHECK(h, hipMemcpyAsync(host_loss, dl, 8, hipMemcpyDeviceToHost, h->stream));
    MLCHECK(h, hipStreamSynchronize(h->stream));
  }
  return 0;
}

lbml_status backward_impl(lbml_net *h, const float *dy, int32_t batch) {
  const Plan &P = h->P;
  const int kb = padded(batch);
  int ping = 0;
  // dZ of the last layer: the caller's FP32 dy (bias gradient) and its BF16
  // operands
  const int nout = P.dims[h->nl];
  MLCHECK(h, to_operands(h->stream, dy, nullptr, batch, nout, h->b(P.off_db[0]), padded(nout), h->b(P.off_dt[0]),
                         P.bp));
  const float *dz = dy;
  for (int l = h->nl - 1; l >= 0; --l) {
    const int din = P.dims[l], dout = P.dims[l + 1];
    // dW[o][i] = sum_b dZ^T[o][b] H^T[i][b]
    GemmArgs gw{};
    gw.A = h->b(P.off_dt[ping]);
    gw.lda = P.bp;
    gw.B = (l == 0) ? h->b(P.off_xt) : h->b(P.off_ht[l - 1]);
    gw.ldb = P.bp;
    gw.M = dout;
    gw.N = din;
    gw.K = kb;
    gw.C = h->f(P.off_g) + P.woff[l];
    gw.ldc = din;
    MLCHECK(h, gemm<EPI_DW>(h->stream, gw));
    hipLaunchKernelGGL(bias_grad_kernel, dim3((dout + 63) / 64), dim3(1024), 0, h->stream, dz, batch, dout,
                       h->f(P.off_g) + P.boff[l]);
    MLCHECK(h, hipGetLastError());
    if (l > 0) {
      // dZ_prev[b][i] = (sum_o dZ[b][o] W[o][i]) SiLU'(Z_prev[b][i])
      GemmArgs gd{};
      gd.A = h->b(P.off_db[ping]);
      gd.lda = padded(dout);
      gd.B = h->pb() + P.wm.wt[l];  // W^T[in][out]: row n = in, K = out
      gd.ldb = padded(dout);
      gd.M = batch;
      gd.N = din;
      gd.K = padded(dout);
      gd.C = h->f(P.off_dz[ping ^ 1]);
      gd.ldc = din;
      gd.Zp = h->f(P.off_z[l - 1]);
      gd.Hb = h->b(P.off_db[ping ^ 1]);
      gd.ldh = padded(din);
      gd.Ht = h->b(P.off_dt[ping ^ 1]);
      gd.ldt = P.bp;
      MLCHECK(h, gemm<EPI_DX>(h->stream, gd));
      dz = gd.C;
      ping ^= 1;
    }
  }
  return 0;
}

bool adam_args_ok(float lr, float b1, float b2, float eps, int32_t t) {
  return t >= 1 && lr > 0 && b1 >= 0 && b1 < 1 && b2 >= 0 && b2 < 1 && eps > 0;
}

lbml_status adam_impl(lbml_net *h, float lr, float b1, float b2, float eps, int32_t t) {
  const long long n = (long long)h->P.params;
  const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
  hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, h->stream, h->f(h->P.off_p),
                     h->f(h->P.off_g), h->f(h->P.off_m), h->f(h->P.off_v), h->pb(), h->P.wm, n, lr, b1, b2, eps,
                     c1, c2);
  MLCHECK(h, hipGetLastError());
  return 0;
}

}  // namespace

extern "C" {

lbml_status lbml_forward(lbml_net *h, const float *x, int32_t batch, float *y) {
  if (!h) return -1;
  if (!x || !y || batch < 1 || batch > h->max_batch) return fail(h, -1, "bad forward arguments");
  return forward_impl(h, x, nullptr, batch, y);
}

lbml_status lbml_mse(lbml_net *h, const float *y, const float *t, int32_t batch, float *dy, double *host_loss) {
  if (!h) return -1;
  if (!y || !t || !dy || batch < 1 || batch > h->max_batch) return fail(h, -1, "bad mse arguments");
  return mse_impl(h, y, t, nullptr, batch, dy, host_loss);
}

lbml_status lbml_backward(lbml_net *h, const float *dy, int32_t batch) {
  if (!h) return -1;
  if (!dy || batch != h->last_batch || batch < 1) return fail(h, -5, "backward needs the forward of this batch");
  return backward_impl(h, dy, batch);
}

lbml_status lbml_adam_step(lbml_net *h, float lr, float b1, float b2, float eps, int32_t t) {
  if (!h) return -1;
  if (!adam_args_ok(lr, b1, b2, eps, t)) return fail(h, -1, "bad Adam arguments");
  return adam_impl(h, lr, b1, b2, eps, t);
}

lbml_status lbml_train_step(lbml_net *h, const float *X, const float *Y, const int32_t *idx, int32_t batch, float lr,
                            float b1, float b2, float eps, int32_t t, double *host_loss) {
  if (!h) return -1;
  if (!X || !Y || !idx || batch < 1 || batch > h->max_batch) return fail(h, -1, "bad train_step arguments");
  if (!adam_args_ok(lr, b1, b2, eps, t)) return fail(h, -1, "bad Adam arguments");
  float *y = h->f(h->P.off_y), *dy = h->f(h->P.off_dy);
  lbml_status st = forward_impl(h, X, idx, batch, y);
  if (st == 0) st = mse_impl(h, y, Y, idx, batch, dy, host_loss);
  if (st == 0) st = backward_impl(h, dy, batch);
  if (st == 0) st = adam_impl(h, lr, b1, b2, eps, t);
  return st;
}

const char *lbml_last_error(const lbml_net *h) { return h ? h->err.c_str() : "NULL handle"; }

}  // extern "C"
