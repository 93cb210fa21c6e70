// Learned edgeMap-variant selector: MLP training kernels (forward, backward,
// Adam), the device-resident inference that picks the next level's variant
// straight from the level counters, and the selector weight store.
//
// Network F=12 -> H=32 (ReLU) -> H=32 (ReLU) -> K=6, FP32, parameters packed as
// W1[F][H] b1[H] W2[H][H] b2[H] W3[H][K] b3[K]. Loss sum(M*(out-Y)^2)/max(sum M,1).
// Gradient sums over samples run in a fixed order (per-chunk partials, then a
// sequential sum over chunks), so training is deterministic.
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "internal.h"
#include "selector_dev.h"

namespace byo {

constexpr int F = BYO_MLP_F, H = BYO_MLP_H, K = BYO_MLP_K, P = BYO_MLP_PARAMS;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + F * H, OFF_W2 = OFF_B1 + H, OFF_B2 = OFF_W2 + H * H,
              OFF_W3 = OFF_B2 + H, OFF_B3 = OFF_W3 + H * K;
static_assert(OFF_B3 + K == P, "parameter layout");

constexpr int MLP_BLOCK = 256;
constexpr int GRAD_CHUNK = 512;   // samples per gradient partial

// ---------------------------------------------------------------- training kernels

// One thread per sample; stores pre-activations z1, z2 ([H][N], sample-minor)
// and outputs out[N][K].
__global__ void __launch_bounds__(MLP_BLOCK) mlp_fwd_kernel(const float *__restrict__ params, const float *__restrict__ X,
                                                            int32_t N, float *__restrict__ out, float *__restrict__ z1s,
                                                            float *__restrict__ z2s) {
  __shared__ float w[P];
  for (int i = threadIdx.x; i < P; i += MLP_BLOCK) w[i] = params[i];
  __syncthreads();
  int64_t n = (int64_t)blockIdx.x * MLP_BLOCK + threadIdx.x;
  if (n >= N) return;
  float x[F], h1[H], h2[H];
#pragma unroll
  for (int i = 0; i < F; ++i) x[i] = X[n * F + i];
#pragma unroll
  for (int j = 0; j < H; ++j) {
    float z = w[OFF_B1 + j];
#pragma unroll
    for (int i = 0; i < F; ++i) z += x[i] * w[OFF_W1 + i * H + j];
    if (z1s) z1s[(int64_t)j * N + n] = z;
    h1[j] = z > 0.f ? z : 0.f;
  }
#pragma unroll
  for (int j = 0; j < H; ++j) {
    float z = w[OFF_B2 + j];
#pragma unroll
    for (int i = 0; i < H; ++i) z += h1[i] * w[OFF_W2 + i * H + j];
    if (z2s) z2s[(int64_t)j * N + n] = z;
    h2[j] = z > 0.f ? z : 0.f;
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    float o = w[OFF_B3 + k];
#pragma unroll
    for (int i = 0; i < H; ++i) o += h2[i] * w[OFF_W3 + i * K + k];
    out[n * K + k] = o;
  }
}

// Loss numerator and mask total in double, one block, fixed order.
__global__ void __launch_bounds__(MLP_BLOCK) mlp_loss_kernel(const float *__restrict__ out, const float *__restrict__ Y,
                                                             const float *__restrict__ M, int64_t NK,
                                                             float *__restrict__ scal /* [0]=den [1]=loss */,
                                                             float *__restrict__ loss_out) {
  double num = 0.0, den = 0.0;
  for (int64_t i = threadIdx.x; i < NK; i += MLP_BLOCK) {
    double r = (double)out[i] - (double)Y[i];
    num += (double)M[i] * r * r;
    den += (double)M[i];
  }
  double tn = block_sum<double, MLP_BLOCK>(num);
  double td = block_sum<double, MLP_BLOCK>(den);
  if (threadIdx.x == 0) {
    double d = td > 1.0 ? td : 1.0;
    scal[0] = (float)d;
    scal[1] = (float)(tn / d);
    if (loss_out) *loss_out = (float)(tn / d);
  }
}

// Per-sample backward: dout[K][N], dz2[H][N], dz1[H][N] (sample-minor).
__global__ void __launch_bounds__(MLP_BLOCK) mlp_bwd_kernel(const float *__restrict__ params, const float *__restrict__ out,
                                                            const float *__restrict__ Y, const float *__restrict__ M,
                                                            int32_t N, const float *__restrict__ scal,
                                                            const float *__restrict__ z1s, const float *__restrict__ z2s,
                                                            float *__restrict__ douts, float *__restrict__ dz2s,
                                                            float *__restrict__ dz1s) {
  __shared__ float w[P];
  for (int i = threadIdx.x; i < P; i += MLP_BLOCK) w[i] = params[i];
  __syncthreads();
  int64_t n = (int64_t)blockIdx.x * MLP_BLOCK + threadIdx.x;
  if (n >= N) return;
  float inv = 2.0f / scal[0];
  float d[K], dz2[H];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    d[k] = M[n * K + k] * (out[n * K + k] - Y[n * K + k]) * inv;
    douts[(int64_t)k * N + n] = d[k];
  }
#pragma unroll
  for (int j = 0; j < H; ++j) {
    float g = 0.f;
#pragma unroll
    for (int k = 0; k < K; ++k) g += d[k] * w[OFF_W3 + j * K + k];
    dz2[j] = z2s[(int64_t)j * N + n] > 0.f ? g : 0.f;
    dz2s[(int64_t)j * N + n] = dz2[j];
  }
#pragma unroll
  for (int i = 0; i < H; ++i) {
    float g = 0.f;
#pragma unroll
    for (int j = 0; j < H; ++j) g += dz2[j] * w[OFF_W2 + i * H + j];
    dz1s[(int64_t)i * N + n] = z1s[(int64_t)i * N + n] > 0.f ? g : 0.f;
  }
}

// Gradient partials: block (p-tile, chunk) sums its chunk's samples for 256 parameters.
__device__ __forceinline__ float grad_term(int p, int64_t n, int32_t N, const float *X, const float *z1s, const float *z2s,
                                          const float *douts, const float *dz2s, const float *dz1s) {
  if (p < OFF_B1) {
    int i = p / H, j = p % H;
    return X[n * F + i] * dz1s[(int64_t)j * N + n];
  }
  if (p < OFF_W2) return dz1s[(int64_t)(p - OFF_B1) * N + n];
  if (p < OFF_B2) {
    int q = p - OFF_W2, i = q / H, j = q % H;
    float a = z1s[(int64_t)i * N + n];
    return (a > 0.f ? a : 0.f) * dz2s[(int64_t)j * N + n];
  }
  if (p < OFF_W3) return dz2s[(int64_t)(p - OFF_B2) * N + n];
  if (p < OFF_B3) {
    int q = p - OFF_W3, i = q / K, k = q % K;
    float a = z2s[(int64_t)i * N + n];
    return (a > 0.f ? a : 0.f) * douts[(int64_t)k * N + n];
  }
  return douts[(int64_t)(p - OFF_B3) * N + n];
}

__global__ void __launch_bounds__(MLP_BLOCK) mlp_grad_partial_kernel(const float *__restrict__ X, int32_t N,
                                                                     const float *__restrict__ z1s,
                                                                     const float *__restrict__ z2s,
                                                                     const float *__restrict__ douts,
                                                                     const float *__restrict__ dz2s,
                                                                     const float *__restrict__ dz1s,
                                                                     float *__restrict__ partial) {
  int p = blockIdx.x * MLP_BLOCK + threadIdx.x;
  int64_t n0 = (int64_t)blockIdx.y * GRAD_CHUNK;
  int64_t n1 = n0 + GRAD_CHUNK < N ? n0 + GRAD_CHUNK : N;
  if (p >= P) return;
  float s = 0.f;
  for (int64_t n = n0; n < n1; ++n) s += grad_term(p, n, N, X, z1s, z2s, douts, dz2s, dz1s);
  partial[(int64_t)blockIdx.y * P + p] = s;
}

__global__ void mlp_grad_reduce_kernel(const float *__restrict__ partial, int32_t chunks, float *__restrict__ grad) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  float s = 0.f;
  for (int c = 0; c < chunks; ++c) s += partial[(int64_t)c * P + p];
  grad[p] = s;
}

__global__ void mlp_adam_kernel(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                                float *__restrict__ v, int32_t t, float lr, float b1, float b2, float eps) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  float gi = g[p];
  float mi = b1 * m[p] + (1.f - b1) * gi;
  float vi = b2 * v[p] + (1.f - b2) * gi * gi;
  m[p] = mi;
  v[p] = vi;
  float mh = mi / (1.f - powf(b1, (float)t));
  float vh = vi / (1.f - powf(b2, (float)t));
  w[p] -= lr * mh / (sqrtf(vh) + eps);
}

struct train_ws {
  int32_t N = -1;
  float *out = nullptr, *z1 = nullptr, *z2 = nullptr, *dout = nullptr, *dz2 = nullptr, *dz1 = nullptr;
  float *partial = nullptr, *scal = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
};

static train_ws g_tw;
static std::mutex g_tw_mu;

static byo_status tw_ensure(int32_t N) {
  if (g_tw.N >= N) return BYO_OK;
  float *ptrs[] = {g_tw.out, g_tw.z1, g_tw.z2, g_tw.dout, g_tw.dz2, g_tw.dz1, g_tw.partial, g_tw.scal, g_tw.grad,
                   g_tw.m, g_tw.v};
  for (float *p : ptrs)
    if (p) (void)hipFree(p);
  g_tw = train_ws();
  int32_t chunks = (N + GRAD_CHUNK - 1) / GRAD_CHUNK;
  BYO_HIP(hipMalloc(&g_tw.out, sizeof(float) * (size_t)N * K));
  BYO_HIP(hipMalloc(&g_tw.z1, sizeof(float) * (size_t)N * H));
  BYO_HIP(hipMalloc(&g_tw.z2, sizeof(float) * (size_t)N * H));
  BYO_HIP(hipMalloc(&g_tw.dout, sizeof(float) * (size_t)N * K));
  BYO_HIP(hipMalloc(&g_tw.dz2, sizeof(float) * (size_t)N * H));
  BYO_HIP(hipMalloc(&g_tw.dz1, sizeof(float) * (size_t)N * H));
  BYO_HIP(hipMalloc(&g_tw.partial, sizeof(float) * (size_t)chunks * P));
  BYO_HIP(hipMalloc(&g_tw.scal, sizeof(float) * 4));
  BYO_HIP(hipMalloc(&g_tw.grad, sizeof(float) * P));
  BYO_HIP(hipMalloc(&g_tw.m, sizeof(float) * P));
  BYO_HIP(hipMalloc(&g_tw.v, sizeof(float) * P));
  g_tw.N = N;
  return BYO_OK;
}

static byo_status loss_grad(const float *params, const float *X, const float *Y, const float *M, int32_t N,
                            float *grad, float *loss, hipStream_t s) {
  BYO_TRY(tw_ensure(N));
  unsigned nb = (unsigned)((N + MLP_BLOCK - 1) / MLP_BLOCK);
  int32_t chunks = (N + GRAD_CHUNK - 1) / GRAD_CHUNK;
  ktimer_scope kt(BYO_K_MLP, s);
  mlp_fwd_kernel<<<nb, MLP_BLOCK, 0, s>>>(params, X, N, g_tw.out, g_tw.z1, g_tw.z2);
  mlp_loss_kernel<<<1, MLP_BLOCK, 0, s>>>(g_tw.out, Y, M, (int64_t)N * K, g_tw.scal, loss);
  mlp_bwd_kernel<<<nb, MLP_BLOCK, 0, s>>>(params, g_tw.out, Y, M, N, g_tw.scal, g_tw.z1, g_tw.z2, g_tw.dout, g_tw.dz2,
                                          g_tw.dz1);
  dim3 gg((P + MLP_BLOCK - 1) / MLP_BLOCK, chunks);
  mlp_grad_partial_kernel<<<gg, MLP_BLOCK, 0, s>>>(X, N, g_tw.z1, g_tw.z2, g_tw.dout, g_tw.dz2, g_tw.dz1, g_tw.partial);
  mlp_grad_reduce_kernel<<<(P + 255) / 256, 256, 0, s>>>(g_tw.partial, chunks, grad);
  BYO_HIP(hipGetLastError());
  return BYO_OK;
}

// ---------------------------------------------------------------- selector store and inference

struct sel_state {
  bool loaded = false;
  int device = -1;
  float *d_w = nullptr;       // params[P], mu[F], sd[F]
  std::vector<float> h_w;     // host copy of d_w for the host-driven level loop
  uint64_t version = 0;       // changes whenever weights are installed or cleared
};
static sel_state g_sel;
static std::mutex g_sel_mu;

struct pick_args {
  float raw[F];
  int32_t allow_pull;
};

// One block of 64 threads: normalise -> MLP -> argmin over the allowed
// variants; -1 if any prediction is not finite.
__global__ void __launch_bounds__(64) mlp_pick_kernel(const float *__restrict__ wts, pick_args a,
                                                      float *__restrict__ pred_out, int32_t *__restrict__ var_out) {
  const int best = sel_pick_block(wts, a.raw, a.allow_pull != 0, pred_out);
  if (threadIdx.x == 0) *var_out = best;
}

bool selector_ready() {
  if (!g_sel.loaded) return false;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  return dev == g_sel.device;
}

const float *selector_device_weights(uint64_t *version) {
  std::lock_guard<std::mutex> lk(g_sel_mu);
  if (version) *version = g_sel.version;
  return selector_ready() ? g_sel.d_w : nullptr;
}

// The host-driven level loop reads each level's counters anyway, so the
// learned choice for the next level is made there: the same float network and
// fallback as mlp_pick_kernel, a few thousand multiply-adds, no launch and no
// extra round trip. Returns -1 when no weights are installed or the
// prediction is not finite (the caller then applies the threshold rule).
int selector_pick_cpu(const level_features &f, bool allow_pull) {
  if (!selector_ready()) return -1;
  const float *w = g_sel.h_w.data();
  float raw[F], x[F], h1[H], h2[H], o[K];
  selector_features((double)f.k, (double)f.degsum, (double)f.unvisited, (double)f.n, (double)f.m, (double)f.max_deg,
                    f.cv, f.dense_in ? 1.0 : 0.0, raw);
  for (int i = 0; i < F; ++i) x[i] = (raw[i] - w[P + i]) / w[P + F + i];
  for (int j = 0; j < H; ++j) {
    float z = w[OFF_B1 + j];
    for (int i = 0; i < F; ++i) z += x[i] * w[OFF_W1 + i * H + j];
    h1[j] = z > 0.f ? z : 0.f;
  }
  for (int j = 0; j < H; ++j) {
    float z = w[OFF_B2 + j];
    for (int i = 0; i < H; ++i) z += h1[i] * w[OFF_W2 + i * H + j];
    h2[j] = z > 0.f ? z : 0.f;
  }
  int best = -1;
  for (int k = 0; k < K; ++k) {
    float z = w[OFF_B3 + k];
    for (int i = 0; i < H; ++i) z += h2[i] * w[OFF_W3 + i * K + k];
    o[k] = z;
    if (!std::isfinite(z)) return -1;
  }
  for (int v = 0; v < K; ++v) {
    bool pull = v == BYO_V_PULL_THREAD || v == BYO_V_PULL_WAVE;
    if (pull && !allow_pull) continue;
    if (best < 0 || o[v] < o[best]) best = v;
  }
  return best;
}

}  // namespace byo

using namespace byo;

extern "C" {

byo_status byo_selector_features(const byo_level_record *r, float *out) {
  BYO_CHECK(r && out, BYO_EINVAL, "null argument");
  selector_features((double)r->k, (double)r->degsum, (double)r->unvisited, (double)r->n, (double)r->m,
                    (double)r->max_deg, r->cv, (double)r->dense_in, out);
  return BYO_OK;
}

int32_t byo_heuristic_choice(int64_t k, int64_t degsum, int64_t m, int64_t max_deg, double cv, const byo_opts *opts,
                             int32_t allow_pull, int64_t max_deg_u) {
  byo_opts o;
  byo_opts_default(&o);
  if (opts) o = *opts;
  return heuristic_rule(k, degsum, m, max_deg, cv, o.dense_divisor, o.t_wave, o.t_block, allow_pull != 0,
                        max_deg_u);
}

byo_status byo_mlp_forward(const float *d_params, const float *d_X, int32_t N, float *d_out, void *stream) {
  BYO_CHECK(d_params && d_X && d_out && N >= 0, BYO_EINVAL, "bad argument");
  if (N == 0) return BYO_OK;
  hipStream_t s = (hipStream_t)stream;
  mlp_fwd_kernel<<<(unsigned)((N + MLP_BLOCK - 1) / MLP_BLOCK), MLP_BLOCK, 0, s>>>(d_params, d_X, N, d_out, nullptr,
                                                                                   nullptr);
  BYO_HIP(hipGetLastError());
  return BYO_OK;
}

byo_status byo_mlp_loss_grad(const float *d_params, const float *d_X, const float *d_Y, const float *d_M, int32_t N,
                             float *d_grad, float *d_loss, void *stream) {
  BYO_CHECK(d_params && d_X && d_Y && d_M && d_grad && N >= 1, BYO_EINVAL, "bad argument");
  std::lock_guard<std::mutex> lk(g_tw_mu);
  return loss_grad(d_params, d_X, d_Y, d_M, N, d_grad, d_loss, (hipStream_t)stream);
}

byo_status byo_mlp_adam(float *d_params, const float *d_grad, float *d_m, float *d_v, int32_t t, float lr, float beta1,
                        float beta2, float eps, void *stream) {
  BYO_CHECK(d_params && d_grad && d_m && d_v && t >= 1, BYO_EINVAL, "bad argument");
  mlp_adam_kernel<<<(P + 255) / 256, 256, 0, (hipStream_t)stream>>>(d_params, d_grad, d_m, d_v, t, lr, beta1, beta2,
                                                                    eps);
  BYO_HIP(hipGetLastError());
  return BYO_OK;
}

byo_status byo_mlp_train(float *d_params, const float *d_X, const float *d_Y, const float *d_M, int32_t N,
                         int32_t steps, float lr, float *d_losses, void *stream) {
  BYO_CHECK(d_params && d_X && d_Y && d_M && N >= 1 && steps >= 0, BYO_EINVAL, "bad argument");
  hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(g_tw_mu);
  BYO_TRY(tw_ensure(N));
  BYO_HIP(hipMemsetAsync(g_tw.m, 0, sizeof(float) * P, s));
  BYO_HIP(hipMemsetAsync(g_tw.v, 0, sizeof(float) * P, s));
  for (int32_t t = 1; t <= steps; ++t) {
    BYO_TRY(loss_grad(d_params, d_X, d_Y, d_M, N, g_tw.grad, d_losses ? d_losses + (t - 1) : nullptr, s));
    mlp_adam_kernel<<<(P + 255) / 256, 256, 0, s>>>(d_params, g_tw.grad, g_tw.m, g_tw.v, t, lr, 0.9f, 0.999f, 1e-8f);
  }
  BYO_HIP(hipGetLastError());
  return BYO_OK;
}

byo_status byo_selector_set(const float *h_params, const float *h_mu, const float *h_sd) {
  BYO_CHECK(h_params && h_mu && h_sd, BYO_EINVAL, "null argument");
  for (int i = 0; i < P; ++i)
    BYO_CHECK(std::isfinite(h_params[i]), BYO_EINVAL, "selector weights contain a non-finite value");
  for (int i = 0; i < F; ++i)
    BYO_CHECK(std::isfinite(h_mu[i]) && std::isfinite(h_sd[i]) && h_sd[i] > 0.f, BYO_EINVAL,
              "feature normalisation must be finite with positive deviations");
  std::lock_guard<std::mutex> lk(g_sel_mu);
  int dev = 0;
  BYO_HIP(hipGetDevice(&dev));
  if (g_sel.d_w && g_sel.device != dev) {
    (void)hipFree(g_sel.d_w);
    g_sel.d_w = nullptr;
  }
  if (!g_sel.d_w) BYO_HIP(hipMalloc(&g_sel.d_w, sizeof(float) * (P + 2 * F)));
  std::vector<float> buf(P + 2 * F);
  std::memcpy(buf.data(), h_params, sizeof(float) * P);
  std::memcpy(buf.data() + P, h_mu, sizeof(float) * F);
  std::memcpy(buf.data() + P + F, h_sd, sizeof(float) * F);
  BYO_HIP(hipMemcpy(g_sel.d_w, buf.data(), sizeof(float) * buf.size(), hipMemcpyHostToDevice));
  g_sel.h_w = buf;
  g_sel.device = dev;
  g_sel.loaded = true;
  ++g_sel.version;
  return BYO_OK;
}

byo_status byo_selector_clear(void) {
  std::lock_guard<std::mutex> lk(g_sel_mu);
  g_sel.loaded = false;
  ++g_sel.version;
  return BYO_OK;
}

byo_status byo_selector_loaded(int32_t *out) {
  BYO_CHECK(out, BYO_EINVAL, "null argument");
  *out = selector_ready() ? 1 : 0;
  return BYO_OK;
}

byo_status byo_selector_predict(const float *h_features, int32_t allow_pull, float *h_pred, int32_t *variant) {
  BYO_CHECK(h_features && variant, BYO_EINVAL, "null argument");
  BYO_CHECK(selector_ready(), BYO_ESTATE, "no selector weights installed on this device");
  pick_args a;
  std::memset(&a, 0, sizeof(a));
  std::memcpy(a.raw, h_features, sizeof(float) * F);
  a.allow_pull = allow_pull ? 1 : 0;
  float *d_pred = nullptr;
  int32_t *d_var = nullptr;
  BYO_HIP(hipMalloc(&d_pred, sizeof(float) * K));
  BYO_HIP(hipMalloc(&d_var, sizeof(int32_t)));
  mlp_pick_kernel<<<1, 64, 0, nullptr>>>(g_sel.d_w, a, d_pred, d_var);
  hipError_t e = hipGetLastError();
  float pred[K];
  int32_t v = -1;
  if (e == hipSuccess) e = hipMemcpy(pred, d_pred, sizeof(pred), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(&v, d_var, sizeof(v), hipMemcpyDeviceToHost);
  (void)hipFree(d_pred);
  (void)hipFree(d_var);
  if (e != hipSuccess) return hip_fail(e, "selector predict", __FILE__, __LINE__);
  if (h_pred) std::memcpy(h_pred, pred, sizeof(pred));
  *variant = v;
  return BYO_OK;
}

}  // extern "C"
