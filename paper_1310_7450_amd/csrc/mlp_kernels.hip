// lbml: the warm-start network (include/lbml.h) on the gfx950 matrix cores.
//
// Every GEMM is C = A B with BF16 operands and FP32 accumulation on
// v_mfma_f32_16x16x16_bf16: one wavefront owns a 16 x 16 tile of C and walks K
// in steps of 16. Operand lanes follow the instruction's layout: lane l holds
// row (l % 16) of A and column (l % 16) of B at k = 4 (l / 16) + 0..3, and
// receives rows 4 (l / 16) + 0..3 of column (l % 16) of C. The epilogues fuse
// the bias, SiLU and the SiLU derivative of the backward pass. Sizes are
// small (batches of a few hundred rows, widths of a few hundred), so the
// kernels favour simplicity over tiling through LDS.
#include "lbml.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16 with round to nearest even (NaN kept quiet).
__host__ __device__ inline unsigned short to_bf16(float f) {
  unsigned int u;
  memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (unsigned short)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

template <typename T>
__device__ inline short operand(const T *p, long long i);
template <>
__device__ inline short operand<float>(const float *p, long long i) {
  return (short)to_bf16(p[i]);
}
template <>
__device__ inline short operand<unsigned short>(const unsigned short *p, long long i) {
  return (short)p[i];
}

__device__ inline float sigmoid(float z) { return 1.0f / (1.0f + expf(-z)); }

enum Epilogue { EPI_NONE = 0, EPI_BIAS = 1, EPI_BIAS_SILU = 2, EPI_SILU_GRAD = 3 };

struct GemmArgs {
  const void *A;
  long long sam, sak;  // A(m, k) = A[m sam + k sak]
  const void *B;
  long long sbk, sbn;  // B(k, n) = B[k sbk + n sbn]
  int M, N, K;
  float *C;
  long long scm, scn;  // C(m, n) = C[m scm + n scn]
  const float *bias;   // EPI_BIAS, EPI_BIAS_SILU: + bias[n]
  float *Z;            // EPI_BIAS_SILU: pre-activation, same layout as C
  const float *Zp;     // EPI_SILU_GRAD: times SiLU'(Zp(m, n)), same layout as C
  int tiles_n;
};

template <typename TA, typename TB, int EPI>
__global__ void __launch_bounds__(64) gemm_kernel(GemmArgs g) {
  const int l = threadIdx.x;
  const int tm = blockIdx.x / g.tiles_n, tn = blockIdx.x % g.tiles_n;
  const int row = tm * 16 + (l & 15);  // A row of this lane
  const int col = tn * 16 + (l & 15);  // B column of this lane
  const int kq = 4 * (l >> 4);
  const TA *A = static_cast<const TA *>(g.A);
  const TB *B = static_cast<const TB *>(g.B);
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < g.K; k0 += 16) {
    bf16x4 a, b;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = k0 + kq + j;
      a[j] = (row < g.M && k < g.K) ? operand<TA>(A, row * g.sam + k * g.sak) : (short)0;
      b[j] = (col < g.N && k < g.K) ? operand<TB>(B, k * g.sbk + col * g.sbn) : (short)0;
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int m = tm * 16 + kq + r, n = col;
    if (m >= g.M || n >= g.N) continue;
    const long long o = m * g.scm + n * g.scn;
    float v = acc[r];
    if (EPI == EPI_BIAS || EPI == EPI_BIAS_SILU) v += g.bias[n];
    if (EPI == EPI_BIAS_SILU) {
      g.Z[o] = v;
      v = v * sigmoid(v);
    }
    if (EPI == EPI_SILU_GRAD) {
      const float z = g.Zp[o], s = sigmoid(z);
      v *= s * (1.0f + z * (1.0f - s));
    }
    g.C[o] = v;
  }
}

// db[n] = sum_m dZ[m][n]
__global__ void bias_grad_kernel(const float *dZ, int M, int N, float *db) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int m = 0; m < M; ++m) s += dZ[(long long)m * N + n];
  db[n] = s;
}

// loss = mean (y - t)^2, dy = 2 (y - t) / count; one workgroup.
__global__ void __launch_bounds__(256) mse_kernel(const float *y, const float *t, long long count, float *dy,
                                                  double *loss) {
  __shared__ double red[256];
  double s = 0.0;
  const float scale = 2.0f / (float)count;
  for (long long i = threadIdx.x; i < count; i += blockDim.x) {
    const float d = y[i] - t[i];
    dy[i] = scale * d;
    s += (double)d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = red[0] / (double)count;
}

__global__ void adam_kernel(float *p, const float *g, float *m, float *v, unsigned short *pb, long long n, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float w = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = w;
  pb[i] = to_bf16(w);
}

__global__ void to_bf16_kernel(const float *p, unsigned short *pb, long long n) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n) pb[i] = to_bf16(p[i]);
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Plan {
  std::vector<int> dims;
  std::vector<size_t> woff, boff;  // parameter offsets (floats)
  size_t params = 0, max_width = 0;
  size_t off_p = 0, off_g = 0, off_m = 0, off_v = 0, off_pb = 0, off_loss = 0, off_dz[2] = {0, 0};
  std::vector<size_t> off_z, off_h;
  size_t bytes = 0;
};

bool make_plan(int nl, const int32_t *dims, int max_batch, Plan &P) {
  if (nl < 1 || !dims || max_batch < 1) return false;
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
  for (int d : P.dims) P.max_width = std::max(P.max_width, (size_t)d);
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
  P.off_pb = take(2 * P.params);
  P.off_loss = take(8);
  P.off_dz[0] = take(4 * (size_t)max_batch * P.max_width);
  P.off_dz[1] = take(4 * (size_t)max_batch * P.max_width);
  for (int l = 0; l < nl; ++l) {
    P.off_z.push_back(take(4 * (size_t)max_batch * P.dims[l + 1]));
    P.off_h.push_back(take(4 * (size_t)max_batch * P.dims[l + 1]));
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
  const float *last_x = nullptr;
  int last_batch = 0;
  std::string err;
  float *f(size_t off) { return reinterpret_cast<float *>(ws + off); }
  unsigned short *pb() { return reinterpret_cast<unsigned short *>(ws + P.off_pb); }
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

template <typename TA, typename TB, int EPI>
hipError_t gemm(hipStream_t s, GemmArgs g) {
  g.tiles_n = (g.N + 15) / 16;
  const int tiles = ((g.M + 15) / 16) * g.tiles_n;
  hipLaunchKernelGGL((gemm_kernel<TA, TB, EPI>), dim3(tiles), dim3(64), 0, s, g);
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
  // zero parameters, gradients and moments (a small fill, not a memset node)
  std::vector<float> zeros(P.params, 0.0f);
  for (size_t off : {P.off_p, P.off_g, P.off_m, P.off_v})
    if (hipMemcpyAsync(h->ws + off, zeros.data(), 4 * P.params, hipMemcpyHostToDevice, h->stream) != hipSuccess) {
      lbml_destroy(h);
      return -3;
    }
  std::vector<unsigned short> zb(P.params, 0);
  if (hipMemcpyAsync(h->ws + P.off_pb, zb.data(), 2 * P.params, hipMemcpyHostToDevice, h->stream) != hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess) {
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
  hipLaunchKernelGGL(to_bf16_kernel, dim3((n + 255) / 256), dim3(256), 0, h->stream, h->f(h->P.off_p), h->pb(),
                     (long long)n);
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

lbml_status lbml_forward(lbml_net *h, const float *x, int32_t batch, float *y) {
  if (!h) return -1;
  if (!x || !y || batch < 1 || batch > h->max_batch) return fail(h, -1, "bad forward arguments");
  const Plan &P = h->P;
  const float *in = x;
  for (int l = 0; l < h->nl; ++l) {
    const int din = P.dims[l], dout = P.dims[l + 1];
    GemmArgs g{};
    g.A = in;
    g.sam = din;
    g.sak = 1;
    g.B = h->pb() + P.woff[l];  // W[o][i] as B(k = i, n = o)
    g.sbk = 1;
    g.sbn = din;
    g.M = batch;
    g.N = dout;
    g.K = din;
    g.scm = dout;
    g.scn = 1;
    g.bias = h->f(P.off_p) + P.boff[l];
    if (l == h->nl - 1) {
      g.C = y;
      MLCHECK(h, (gemm<float, unsigned short, EPI_BIAS>(h->stream, g)));
    } else {
      g.C = h->f(P.off_h[l]);
      g.Z = h->f(P.off_z[l]);
      MLCHECK(h, (gemm<float, unsigned short, EPI_BIAS_SILU>(h->stream, g)));
      in = g.C;
    }
  }
  h->last_x = x;
  h->last_batch = batch;
  return 0;
}

lbml_status lbml_mse(lbml_net *h, const float *y, const float *t, int32_t batch, float *dy, double *host_loss) {
  if (!h) return -1;
  if (!y || !t || !dy || batch < 1 || batch > h->max_batch) return fail(h, -1, "bad mse arguments");
  const long long count = (long long)batch * h->P.dims[h->nl];
  double *dl = reinterpret_cast<double *>(h->ws + h->P.off_loss);
  hipLaunchKernelGGL(mse_kernel, dim3(1), dim3(256), 0, h->stream, y, t, count, dy, dl);
  MLCHECK(h, hipGetLastError());
  if (host_loss) {
    MLCHECK(h, hipMemcpyAsync(host_loss, dl, 8, hipMemcpyDeviceToHost, h->stream));
    MLCHECK(h, hipStreamSynchronize(h->stream));
  }
  return 0;
}

lbml_status lbml_backward(lbml_net *h, const float *dy, int32_t batch) {
  if (!h) return -1;
  if (!dy || batch != h->last_batch || !h->last_x) return fail(h, -5, "backward needs the forward of this batch");
  const Plan &P = h->P;
  const float *dz = dy;  // gradient of the current layer's pre-activation
  int ping = 0;
  for (int l = h->nl - 1; l >= 0; --l) {
    const int din = P.dims[l], dout = P.dims[l + 1];
    const float *hin = (l == 0) ? h->last_x : h->f(P.off_h[l - 1]);
    // dW[o][i] = sum_b dz[b][o] hin[b][i]
    GemmArgs gw{};
    gw.A = dz;
    gw.sam = 1;
    gw.sak = dout;
    gw.B = hin;
    gw.sbk = din;
    gw.sbn = 1;
    gw.M = dout;
    gw.N = din;
    gw.K = batch;
    gw.C = h->f(P.off_g) + P.woff[l];
    gw.scm = din;
    gw.scn = 1;
    MLCHECK(h, (gemm<float, float, EPI_NONE>(h->stream, gw)));
    hipLaunchKernelGGL(bias_grad_kernel, dim3((dout + 255) / 256), dim3(256), 0, h->stream, dz, batch, dout,
                       h->f(P.off_g) + P.boff[l]);
    MLCHECK(h, hipGetLastError());
    if (l > 0) {
      // dz_prev[b][i] = (sum_o dz[b][o] W[o][i]) * SiLU'(z_prev[b][i])
      GemmArgs gd{};
      gd.A = dz;
      gd.sam = dout;
      gd.sak = 1;
      gd.B = h->pb() + P.woff[l];
      gd.sbk = din;
      gd.sbn = 1;
      gd.M = batch;
      gd.N = din;
      gd.K = dout;
      gd.C = h->f(P.off_dz[ping]);
      gd.scm = din;
      gd.scn = 1;
      gd.Zp = h->f(P.off_z[l - 1]);
      MLCHECK(h, (gemm<float, unsigned short, EPI_SILU_GRAD>(h->stream, gd)));
      dz = gd.C;
      ping ^= 1;
    }
  }
  return 0;
}

lbml_status lbml_adam_step(lbml_net *h, float lr, float b1, float b2, float eps, int32_t t) {
  if (!h) return -1;
  if (t < 1 || !(lr > 0) || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1) || !(eps > 0))
    return fail(h, -1, "bad Adam arguments");
  const long long n = (long long)h->P.params;
  const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
  hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, h->stream, h->f(h->P.off_p),
                     h->f(h->P.off_g), h->f(h->P.off_m), h->f(h->P.off_v), h->pb(), n, lr, b1, b2, eps, c1, c2);
  MLCHECK(h, hipGetLastError());
  return 0;
}

const char *lbml_last_error(const lbml_net *h) { return h ? h->err.c_str() : "NULL handle"; }

}  // extern "C"
