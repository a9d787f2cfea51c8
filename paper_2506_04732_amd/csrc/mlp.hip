// Learned warm start: a small multilayer perceptron (tanh hidden layers,
// linear output) that maps an instance's parameters to TT cores, its
// training (backward pass, Adam), the gauge-invariant TT fitting loss, BF16
// inference, and the packing of TT cores to and from the network's flat
// output vector.  All FP32 on the device; the dense layers use the library's
// FP32 GEMM (the layers are 256 wide: no shape here is large enough to pay
// for a matrix-core path).
#include "mlp.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <random>

namespace t2s2 {

namespace {

constexpr int kB = 256;

inline int grid_of(long n) { return (int)std::max<long>(1, std::min<long>((n + kB - 1) / kB, 4096)); }

__global__ void bias_act_kernel(long B, int w, float* __restrict__ Z, const float* __restrict__ b, int act) {
  const long n = B * w;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const float z = Z[e] + b[e % w];
    Z[e] = act ? tanhf(z) : z;
  }
}

// G *= 1 - H^2 (derivative of tanh through its output)
__global__ void tanh_back_kernel(long n, float* __restrict__ G, const float* __restrict__ H) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const float h = H[e];
    G[e] *= 1.0f - h * h;
  }
}

// db[j] = sum_b G[b, j]  (fixed summation order)
__global__ void colsum_kernel(int B, int w, const float* __restrict__ G, float* __restrict__ db) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= w) return;
  float s = 0.0f;
  for (int b = 0; b < B; ++b) s += G[(long)b * w + j];
  db[j] = s;
}

__global__ void adam_kernel(long n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, float lr, float b1, float b2, float eps, float bc1, float bc2) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const float ge = g[e];
    const float me = b1 * m[e] + (1.0f - b1) * ge;
    const float ve = b2 * v[e] + (1.0f - b2) * ge * ge;
    m[e] = me;
    v[e] = ve;
    p[e] -= lr * (me / bc1) / (sqrtf(ve / bc2) + eps);
  }
}

__global__ void gather_rows_kernel(int rows, int w, const float* __restrict__ src, const int* __restrict__ idx,
                                   float* __restrict__ dst) {
  const long n = (long)rows * w;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const long r = e / w;
    dst[e] = src[(long)idx[r] * w + e % w];
  }
}

// out[j] = mean_r in[r, j] (fixed summation order)
__global__ void col_mean_kernel(int rows, int w, const float* __restrict__ in, float* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= w) return;
  double s = 0.0;
  for (int r = 0; r < rows; ++r) s += in[(long)r * w + j];
  out[j] = (float)(s / rows);
}

__global__ void scale_kernel(long n, float* __restrict__ x, float s) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) x[e] *= s;
}

// ---- BF16: round to nearest even (NaN kept quiet), and back
__device__ inline unsigned short f32_to_bf16(float f) {
  unsigned int u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (unsigned short)((u >> 16) | 0x0040u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ inline float bf16_to_f32(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

__global__ void to_bf16_kernel(long n, const float* __restrict__ x, unsigned short* __restrict__ y) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    y[e] = f32_to_bf16(x[e]);
}

// Y[b, j] = act(sum_i W[j, i] X[b, i] + bias[j]) with BF16 W and bias, FP32
// inputs and accumulation; one wavefront per output row j (lanes stride i).
__global__ void __launch_bounds__(256) linear_bf16_kernel(int B, int win, int wout,
                                                          const unsigned short* __restrict__ W,
                                                          const unsigned short* __restrict__ bias,
                                                          const float* __restrict__ X, float* __restrict__ Y,
                                                          int act) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= wout) return;
  const unsigned short* wr = W + (long)j * win;
  const float bj = bf16_to_f32(bias[j]);
  for (int b = 0; b < B; ++b) {
    const float* xr = X + (long)b * win;
    float s = 0.0f;
    for (int i = lane; i < win; i += 64) s = fmaf(bf16_to_f32(wr[i]), xr[i], s);
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) {
      const float z = s + bj;
      Y[(long)b * wout + j] = act ? tanhf(z) : z;
    }
  }
}

// ---- gauge-invariant TT fitting loss: one workgroup per sample.
// Flat vector = cores of uniform interior rank r (boundary ranks 1), core l
// [r_l][n_l][r_{l+1}] at offset off[l].  Environments E (left) and F
// (right) are r x r blocks with row stride r; E_0 = F_d = 1.
struct TTShape {
  int d, r, total;
  int n[16];
  int off[17];
};

__device__ inline int rk(const TTShape& s, int l) { return (l == 0 || l == s.d) ? 1 : s.r; }

// E_{l+1}[b, c] = sum_{a, a', i} A_l[a, i, b] E_l[a, a'] B_l[a', i, c]
__device__ void left_step(const TTShape& s, int l, const float* A, const float* Bc, const float* E, float* En) {
  const int r0 = rk(s, l), r1 = rk(s, l + 1), n = s.n[l], r = s.r;
  for (int e = threadIdx.x; e < r1 * r1; e += blockDim.x) {
    const int b = e / r1, c = e % r1;
    float acc = 0.0f;
    for (int a = 0; a < r0; ++a)
      for (int i = 0; i < n; ++i) {
        const float x = A[(a * n + i) * r1 + b];
        float y = 0.0f;
        for (int a2 = 0; a2 < r0; ++a2) y = fmaf(E[a * r + a2], Bc[(a2 * n + i) * r1 + c], y);
        acc = fmaf(x, y, acc);
      }
    En[b * r + c] = acc;
  }
}

// F_l[a, c] = sum_{b, b', i} A_l[a, i, b] F_{l+1}[b, b'] B_l[c, i, b']
__device__ void right_step(const TTShape& s, int l, const float* A, const float* Bc, const float* F, float* Fn) {
  const int r0 = rk(s, l), r1 = rk(s, l + 1), n = s.n[l], r = s.r;
  for (int e = threadIdx.x; e < r0 * r0; e += blockDim.x) {
    const int a = e / r0, c = e % r0;
    float acc = 0.0f;
    for (int i = 0; i < n; ++i)
      for (int b = 0; b < r1; ++b) {
        const float x = A[(a * n + i) * r1 + b];
        float y = 0.0f;
        for (int b2 = 0; b2 < r1; ++b2) y = fmaf(F[b * r + b2], Bc[(c * n + i) * r1 + b2], y);
        acc = fmaf(x, y, acc);
      }
    Fn[a * r + c] = acc;
  }
}

__global__ void __launch_bounds__(256) tt_fit_loss_kernel(TTShape s, const float* __restrict__ pred,
                                                          const float* __restrict__ target,
                                                          float* __restrict__ loss, float* __restrict__ dpred,
                                                          float gscale) {
  extern __shared__ __align__(16) float sm[];
  const int tot = s.total, d = s.d, r = s.r, rr = r * r;
  float* P = sm;
  float* T = P + tot;
  float* Lpp = T + tot;
  float* Lpt = Lpp + (d + 1) * rr;
  float* Ltt = Lpt + (d + 1) * rr;
  float* Rpp = Ltt + (d + 1) * rr;
  float* Rpt = Rpp + (d + 1) * rr;
  const long base = (long)blockIdx.x * tot;
  for (int e = threadIdx.x; e < tot; e += blockDim.x) {
    P[e] = pred[base + e];
    T[e] = target[base + e];
  }
  if (threadIdx.x == 0) {
    Lpp[0] = Lpt[0] = Ltt[0] = 1.0f;
    Rpp[d * rr] = Rpt[d * rr] = 1.0f;
  }
  __syncthreads();
  for (int l = 0; l < d; ++l) {
    const float* Pl = P + s.off[l];
    const float* Tl = T + s.off[l];
    left_step(s, l, Pl, Pl, Lpp + l * rr, Lpp + (l + 1) * rr);
    left_step(s, l, Pl, Tl, Lpt + l * rr, Lpt + (l + 1) * rr);
    left_step(s, l, Tl, Tl, Ltt + l * rr, Ltt + (l + 1) * rr);
    __syncthreads();
  }
  for (int l = d - 1; l >= 0; --l) {
    const float* Pl = P + s.off[l];
    const float* Tl = T + s.off[l];
    right_step(s, l, Pl, Pl, Rpp + (l + 1) * rr, Rpp + l * rr);
    right_step(s, l, Pl, Tl, Rpt + (l + 1) * rr, Rpt + l * rr);
    __syncthreads();
  }
  const float pp = Lpp[d * rr], pt = Lpt[d * rr], tt = Ltt[d * rr];
  if (threadIdx.x == 0) loss[blockIdx.x] = (pp - 2.0f * pt + tt) / tt;
  // dloss/dP_l[a, i, b] = (2 sum Lpp_l[a,c] P_l[c,i,e] Rpp_{l+1}[b,e] - 2 sum Lpt_l[a,c] T_l[c,i,e] Rpt_{l+1}[b,e]) / tt
  const float sc = 2.0f * gscale / tt;
  for (int l = 0; l < d; ++l) {
    const int r0 = rk(s, l), r1 = rk(s, l + 1), n = s.n[l];
    const float* Pl = P + s.off[l];
    const float* Tl = T + s.off[l];
    const float* Lp = Lpp + l * rr;
    const float* Lt = Lpt + l * rr;
    const float* Rp = Rpp + (l + 1) * rr;
    const float* Rt = Rpt + (l + 1) * rr;
    for (int e = threadIdx.x; e < r0 * n * r1; e += blockDim.x) {
      const int a = e / (n * r1), i = (e / r1) % n, b = e % r1;
      float gp = 0.0f, gt = 0.0f;
      for (int c = 0; c < r0; ++c) {
        float yp = 0.0f, yt = 0.0f;
        for (int f = 0; f < r1; ++f) {
          yp = fmaf(Pl[(c * n + i) * r1 + f], Rp[b * r + f], yp);
          yt = fmaf(Tl[(c * n + i) * r1 + f], Rt[b * r + f], yt);
        }
        gp = fmaf(Lp[a * r + c], yp, gp);
        gt = fmaf(Lt[a * r + c], yt, gt);
      }
      dpred[base + s.off[l] + e] = sc * (gp - gt);
    }
  }
}

// ---- packing between FP64 TT cores (ranks <= r) and the flat FP32 vector.
// With canonical signs, the sign of every rank column of cores 0..d-2 is
// chosen so that its entry of largest magnitude is positive (the flip is
// undone in the next core's matching row, so the tensor is unchanged).
struct PackArgs {
  int d, r, canon;
  int n[16];
  int xr[17];
  int off[17];
  const double* core[16];
};

__global__ void __launch_bounds__(256) tt_pack_kernel(PackArgs a, float* __restrict__ out) {
  __shared__ float sgn_in[64], sgn_out[64];
  __shared__ float red_v[256];
  __shared__ int red_i[256];
  if (threadIdx.x < 64) sgn_in[threadIdx.x] = 1.0f;
  __syncthreads();
  for (int l = 0; l < a.d; ++l) {
    const int r0 = a.xr[l], r1 = a.xr[l + 1], n = a.n[l];
    const int R0 = (l == 0) ? 1 : a.r, R1 = (l == a.d - 1) ? 1 : a.r;
    const double* c = a.core[l];
    // column signs
    for (int b = 0; b < r1; ++b) {
      float best = -1.0f;
      int bi = 0;
      for (int e = threadIdx.x; e < r0 * n; e += blockDim.x) {
        const float v = fabsf((float)c[(long)e * r1 + b]);
        if (v > best) { best = v; bi = e; }
      }
      red_v[threadIdx.x] = best;
      red_i[threadIdx.x] = bi;
      __syncthreads();
      if (threadIdx.x == 0) {
        float bv = -1.0f;
        int bx = 0;
        for (int t = 0; t < (int)blockDim.x; ++t)
          if (red_v[t] > bv || (red_v[t] == bv && red_i[t] < bx)) { bv = red_v[t]; bx = red_i[t]; }
        const int a0 = bx / n;
        const float v = (float)c[(long)bx * r1 + b] * sgn_in[a0];
        sgn_out[b] = (a.canon && l < a.d - 1 && v < 0.0f) ? -1.0f : 1.0f;
      }
      __syncthreads();
    }
    for (int e = threadIdx.x; e < R0 * n * R1; e += blockDim.x) {
      const int p = e / (n * R1), i = (e / R1) % n, q = e % R1;
      float v = 0.0f;
      if (p < r0 && q < r1) v = (float)c[((long)p * n + i) * r1 + q] * sgn_in[p] * sgn_out[q];
      out[a.off[l] + e] = v;
    }
    __syncthreads();
    if (threadIdx.x < 64) sgn_in[threadIdx.x] = (threadIdx.x < r1) ? sgn_out[threadIdx.x] : 1.0f;
    __syncthreads();
  }
}

__global__ void unpack_kernel(long n, const float* __restrict__ in, double* __restrict__ out) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    out[e] = (double)in[e];
}

}  // namespace

// ============================================================== network
long mlp_param_count(const std::vector<int>& w) {
  long t = 0;
  for (size_t k = 0; k + 1 < w.size(); ++k) t += (long)w[k + 1] * w[k] + w[k + 1];
  return t;
}

Mlp::~Mlp() {
  for (void* p : {(void*)params, (void*)grad, (void*)m, (void*)v, (void*)params16})
    if (p) (void)hipFree(p);
}

Mlp* mlp_create(const std::vector<int>& widths, unsigned long long seed) {
  T2S2_CHECK(widths.size() >= 2 && widths.size() <= 16, "mlp: need 1 to 15 layers");
  for (int w : widths) T2S2_CHECK(w >= 1 && w <= 65536, "mlp: widths must be in [1, 65536]");
  Mlp* N = new Mlp();
  try {
    N->w = widths;
    N->nparam = mlp_param_count(widths);
    const size_t bytes = (size_t)N->nparam * sizeof(float);
    T2S2_HIP(hipMalloc(&N->params, bytes));
    T2S2_HIP(hipMalloc(&N->grad, bytes));
    T2S2_HIP(hipMalloc(&N->m, bytes));
    T2S2_HIP(hipMalloc(&N->v, bytes));
    T2S2_HIP(hipMalloc(&N->params16, (size_t)N->nparam * sizeof(unsigned short)));
    // Glorot-uniform weights, zero biases (seeded host generator)
    std::vector<float> h((size_t)N->nparam, 0.0f);
    std::mt19937_64 rng(seed);
    long o = 0;
    for (size_t k = 0; k + 1 < widths.size(); ++k) {
      const int wi = widths[k], wo = widths[k + 1];
      const double lim = std::sqrt(6.0 / (wi + wo));
      std::uniform_real_distribution<double> U(-lim, lim);
      for (long e = 0; e < (long)wo * wi; ++e) h[o + e] = (float)U(rng);
      o += (long)wo * wi + wo;
    }
    T2S2_HIP(hipMemcpy(N->params, h.data(), bytes, hipMemcpyHostToDevice));
    T2S2_HIP(hipMemset(N->m, 0, bytes));
    T2S2_HIP(hipMemset(N->v, 0, bytes));
    T2S2_HIP(hipMemset(N->grad, 0, bytes));
  } catch (...) {
    delete N;
    throw;
  }
  return N;
}

static float* act_buf(Mlp& N, int B, int k) {
  // activations H_1 .. H_{L-1} for the last forward pass (batch B)
  long o = 0;
  for (int j = 1; j < k; ++j) o += (long)B * N.w[j];
  return N.sc.get<float>("mlp.acts", (size_t)B * std::accumulate(N.w.begin() + 1, N.w.end() - 1, 0L) + 1) + o;
}

void mlp_forward(Mlp& N, hipStream_t s, int B, const float* X, float* Y) {
  T2S2_CHECK(B >= 1, "mlp: batch must be >= 1");
  const int L = (int)N.w.size() - 1;
  const float* H = X;
  long o = 0;
  for (int k = 0; k < L; ++k) {
    const int wi = N.w[k], wo = N.w[k + 1];
    const float* W = N.params + o;
    const float* b = W + (long)wo * wi;
    o += (long)wo * wi + wo;
    float* Z = (k < L - 1) ? act_buf(N, B, k + 1) : Y;
    gemm<float>(s, OpN, OpT, B, wo, wi, 1.0f, H, wi, 0, W, wi, 0, 0.0f, Z, wo, 0, 1);
    hipLaunchKernelGGL(bias_act_kernel, dim3(grid_of((long)B * wo)), dim3(kB), 0, s, (long)B, wo, Z, b,
                       k < L - 1 ? 1 : 0);
    T2S2_LAUNCH_CHECK();
    H = Z;
  }
  N.last_batch = B;
}

void mlp_backward(Mlp& N, hipStream_t s, int B, const float* X, const float* dY) {
  T2S2_CHECK(B == N.last_batch, "mlp: backward needs the forward pass of the same batch just before");
  const int L = (int)N.w.size() - 1;
  std::vector<long> off(L + 1, 0);
  for (int k = 0; k < L; ++k) off[k + 1] = off[k] + (long)N.w[k + 1] * N.w[k] + N.w[k + 1];
  const int wmax = *std::max_element(N.w.begin(), N.w.end());
  float* G0 = N.sc.get<float>("mlp.g0", (size_t)B * wmax);
  float* G1 = N.sc.get<float>("mlp.g1", (size_t)B * wmax);
  const float* G = dY;
  for (int k = L - 1; k >= 0; --k) {
    const int wi = N.w[k], wo = N.w[k + 1];
    const float* Hk = (k == 0) ? X : act_buf(N, B, k);
    float* dW = N.grad + off[k];
    float* db = dW + (long)wo * wi;
    gemm<float>(s, OpT, OpN, wo, wi, B, 1.0f, G, wo, 0, Hk, wi, 0, 0.0f, dW, wi, 0, 1);
    hipLaunchKernelGGL(colsum_kernel, dim3((wo + 255) / 256), dim3(256), 0, s, B, wo, G, db);
    T2S2_LAUNCH_CHECK();
    if (k > 0) {
      float* Gn = (G == G0) ? G1 : G0;
      gemm<float>(s, OpN, OpN, B, wi, wo, 1.0f, G, wo, 0, N.params + off[k], wi, 0, 0.0f, Gn, wi, 0, 1);
      hipLaunchKernelGGL(tanh_back_kernel, dim3(grid_of((long)B * wi)), dim3(kB), 0, s, (long)B * wi, Gn, Hk);
      T2S2_LAUNCH_CHECK();
      G = Gn;
    }
  }
}

void mlp_adam(Mlp& N, hipStream_t s, float lr, float b1, float b2, float eps) {
  N.t += 1;
  const float bc1 = 1.0f - std::pow(b1, (float)N.t), bc2 = 1.0f - std::pow(b2, (float)N.t);
  hipLaunchKernelGGL(adam_kernel, dim3(grid_of(N.nparam)), dim3(kB), 0, s, N.nparam, N.params, N.grad, N.m, N.v, lr,
                     b1, b2, eps, bc1, bc2);
  T2S2_LAUNCH_CHECK();
  N.bf16_valid = false;
}

void mlp_infer_bf16(Mlp& N, hipStream_t s, int B, const float* X, float* Y) {
  T2S2_CHECK(B >= 1, "mlp: batch must be >= 1");
  if (!N.bf16_valid) {
    hipLaunchKernelGGL(to_bf16_kernel, dim3(grid_of(N.nparam)), dim3(kB), 0, s, N.nparam, N.params, N.params16);
    T2S2_LAUNCH_CHECK();
    N.bf16_valid = true;
  }
  const int L = (int)N.w.size() - 1;
  const int wmax = *std::max_element(N.w.begin(), N.w.end());
  float* A0 = N.sc.get<float>("mlp.i0", (size_t)B * wmax);
  float* A1 = N.sc.get<float>("mlp.i1", (size_t)B * wmax);
  const float* H = X;
  long o = 0;
  for (int k = 0; k < L; ++k) {
    const int wi = N.w[k], wo = N.w[k + 1];
    float* Z = (k == L - 1) ? Y : ((H == A0) ? A1 : A0);
    hipLaunchKernelGGL(linear_bf16_kernel, dim3((wo + 3) / 4), dim3(256), 0, s, B, wi, wo, N.params16 + o,
                       N.params16 + o + (long)wo * wi, H, Z, k < L - 1 ? 1 : 0);
    T2S2_LAUNCH_CHECK();
    o += (long)wo * wi + wo;
    H = Z;
  }
}

static TTShape make_shape(int d, const int* n, int r) {
  T2S2_CHECK(d >= 1 && d <= 16 && r >= 1 && r <= 16, "tt fit: need 1 <= d <= 16 and 1 <= rank <= 16");
  TTShape s{};
  s.d = d;
  s.r = r;
  int o = 0;
  for (int l = 0; l < d; ++l) {
    T2S2_CHECK(n[l] >= 1 && n[l] <= 64, "tt fit: mode sizes must be in [1, 64]");
    s.n[l] = n[l];
    s.off[l] = o;
    o += ((l == 0) ? 1 : r) * n[l] * ((l == d - 1) ? 1 : r);
  }
  s.off[d] = o;
  s.total = o;
  return s;
}

int tt_flat_size(int d, const int* n, int r) { return make_shape(d, n, r).total; }

void tt_fit_loss(hipStream_t s, int B, int d, const int* n, int r, const float* pred, const float* target,
                 float* loss, float* dpred, float gscale) {
  const TTShape sh = make_shape(d, n, r);
  const size_t lds = ((size_t)2 * sh.total + 5 * (size_t)(d + 1) * r * r) * sizeof(float);
  T2S2_CHECK(lds <= 160000, "tt fit: cores and environments exceed the 160 KB of LDS of one workgroup");
  if (B <= 0) return;
  hipLaunchKernelGGL(tt_fit_loss_kernel, dim3(B), dim3(256), lds, s, sh, pred, target, loss, dpred, gscale);
  T2S2_LAUNCH_CHECK();
}

std::vector<float> mlp_train(Mlp& N, hipStream_t s, int count, const float* X, const float* Yt, int d, const int* n,
                             int r, int epochs, int batch, float lr, unsigned long long seed) {
  const int win = N.w.front(), wout = N.w.back();
  T2S2_CHECK(tt_flat_size(d, n, r) == wout, "mlp train: output width must equal the flat TT size");
  T2S2_CHECK(count >= 1 && epochs >= 0 && batch >= 1, "mlp train: bad count, epochs or batch");
  batch = std::min(batch, count);
  float* xb = N.sc.get<float>("tr.x", (size_t)batch * win);
  float* yb = N.sc.get<float>("tr.y", (size_t)batch * wout);
  float* tb = N.sc.get<float>("tr.t", (size_t)batch * wout);
  float* dy = N.sc.get<float>("tr.dy", (size_t)batch * wout);
  float* lossd = N.sc.get<float>("tr.loss", (size_t)count);
  int* idxd = N.sc.get<int>("tr.idx", (size_t)count);
  std::vector<int> idx(count);
  std::iota(idx.begin(), idx.end(), 0);
  std::mt19937_64 rng(seed);
  std::vector<float> hist;
  std::vector<float> hl(count);
  if (N.t == 0) {
    // untrained network: start from the mean target (output bias) with the
    // output weights shrunk tenfold, so that the first prediction is a
    // typical TT rather than the near-zero output of random weights, whose
    // multilinear gradients would vanish
    const int L = (int)N.w.size() - 1;
    long o = 0;
    for (int k = 0; k + 1 < L; ++k) o += (long)N.w[k + 1] * N.w[k] + N.w[k + 1];
    float* Wout = N.params + o;
    const long nw = (long)N.w[L] * N.w[L - 1];
    hipLaunchKernelGGL(scale_kernel, dim3(grid_of(nw)), dim3(kB), 0, s, nw, Wout, 0.1f);
    hipLaunchKernelGGL(col_mean_kernel, dim3((wout + 255) / 256), dim3(256), 0, s, count, wout, Yt, Wout + nw);
    T2S2_LAUNCH_CHECK();
    N.bf16_valid = false;
  }
  for (int ep = 0; ep < epochs; ++ep) {
    std::shuffle(idx.begin(), idx.end(), rng);
    T2S2_HIP(hipMemcpyAsync(idxd, idx.data(), sizeof(int) * count, hipMemcpyHostToDevice, s));
    for (int b0 = 0; b0 < count; b0 += batch) {
      const int B = std::min(batch, count - b0);
      hipLaunchKernelGGL(gather_rows_kernel, dim3(grid_of((long)B * win)), dim3(kB), 0, s, B, win, X, idxd + b0, xb);
      hipLaunchKernelGGL(gather_rows_kernel, dim3(grid_of((long)B * wout)), dim3(kB), 0, s, B, wout, Yt, idxd + b0,
                         tb);
      T2S2_LAUNCH_CHECK();
      mlp_forward(N, s, B, xb, yb);
      // mean loss over the batch: gradient scaled by 1 / B
      tt_fit_loss(s, B, d, n, r, yb, tb, lossd + b0, dy, 1.0f / (float)B);
      mlp_backward(N, s, B, xb, dy);
      mlp_adam(N, s, lr, 0.9f, 0.999f, 1e-8f);
    }
    T2S2_HIP(hipMemcpyAsync(hl.data(), lossd, sizeof(float) * count, hipMemcpyDeviceToHost, s));
    T2S2_HIP(hipStreamSynchronize(s));
    double sum = 0.0;
    for (float v : hl) sum += v;
    hist.push_back((float)(sum / count));
  }
  return hist;
}

void tt_pack(hipStream_t s, const DTT& x, int r, int canonical, float* out) {
  T2S2_CHECK(x.d >= 1 && x.d <= 16 && r >= 1 && r <= 16, "tt pack: need 1 <= d <= 16, 1 <= rank <= 16");
  PackArgs a{};
  a.d = x.d;
  a.r = r;
  a.canon = canonical;
  int o = 0;
  for (int l = 0; l < x.d; ++l) {
    T2S2_CHECK(x.r[l + 1] <= r && x.r[l] <= r, "tt pack: TT ranks exceed the packed rank");
    T2S2_CHECK(x.n[l] >= 1 && x.n[l] <= 64, "tt pack: mode sizes must be in [1, 64]");
    a.n[l] = x.n[l];
    a.core[l] = x.c[l];
    a.off[l] = o;
    o += ((l == 0) ? 1 : r) * x.n[l] * ((l == x.d - 1) ? 1 : r);
  }
  for (int l = 0; l <= x.d; ++l) a.xr[l] = x.r[l];
  hipLaunchKernelGGL(tt_pack_kernel, dim3(1), dim3(256), 0, s, a, out);
  T2S2_LAUNCH_CHECK();
}

void tt_unpack(hipStream_t s, int d, const int* n, int r, const float* in, DTT& x) {
  const TTShape sh = make_shape(d, n, r);
  x.d = d;
  x.n.assign(n, n + d);
  x.r.assign(d + 1, r);
  x.r[0] = x.r[d] = 1;
  for (int l = 0; l < d; ++l) {
    const long sz = (long)x.r[l] * n[l] * x.r[l + 1];
    hipLaunchKernelGGL(unpack_kernel, dim3(grid_of(sz)), dim3(kB), 0, s, sz, in + sh.off[l], x.c[l]);
    T2S2_LAUNCH_CHECK();
  }
}

}  // namespace t2s2
