// trs_mlp.hip -- the frontier predictor on the device: batched forward and
// backward passes, the Adam step, the compiled decision table, and their
// C-ABI entry points.
//
// The network (a learned component of this library; the paper has none):
//   x  = [E[sym] (16), arity/8, c_0..c_4, bucket(age)/15, 0]        (24)
//   h1 = relu(W1 x + b1) (32);  h2 = relu(W2 h1 + b2) (32)
//   z  = w3 . h2 + b3;  p = sigmoid(z);  loss = mean(softplus(z) - y z)
// Weights are bfloat16, every sum accumulates in float32.  Training keeps
// float32 master weights and rounds them to bfloat16 after every step.
//
// One workgroup of 256 threads takes tiles of 64 records; the weights and
// the tile's activations live in LDS.  Each thread owns fixed gradient
// entries and accumulates them in registers over all its tiles, so a launch
// issues one global atomic per parameter per workgroup.  The contractions
// are 64 x 24 x 32 and 64 x 32 x 32 per tile: far too small for matrix
// cores to pay, so they are plain FP32 FMAs.
//
// The decision table: the input space is finite (symbol, 5 bits, 16 age
// buckets), so the network is evaluated once on every input -- by the same
// forward code -- and the keep decisions p >= threshold are packed into a
// bit table that the round kernel holds in LDS.  A lookup gives exactly the
// decision a per-node evaluation would.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "trs.h"
#include "trs_mlp.h"

namespace {

#define T_TILE 64
#define NT 256
constexpr int EMB = TRS_MLP_EMB, DIN = TRS_MLP_DIN, H = TRS_MLP_H;

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ uint16_t f2bf(float f) {
  // round to nearest, ties to even (finite values)
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Forward (and, with want_grad, backward) pass over records [0, n).
// Accumulates scale * d(sum of losses)/d(param) into grad, the summed loss
// into *loss, and p per record into probs (if not null).
__global__ void __launch_bounds__(NT) k_mlp_grad(const uint16_t *__restrict__ wbf, int n_sym,
                                                 const uint64_t *__restrict__ rec, long long n,
                                                 float scale, float *grad, float *loss,
                                                 float *probs, int want_grad) {
  __shared__ float W1[H * DIN], b1[H], W2[H * H], b2[H], w3[H];
  __shared__ float X[T_TILE * DIN], H1[T_TILE * H], H2[T_TILE * H], D[T_TILE * H];
  __shared__ float DZ[T_TILE], Y[T_TILE];
  __shared__ int SYM[T_TILE];
  __shared__ float b3s, lsum;
  const int tid = threadIdx.x;
  const int oW1 = EMB * n_sym, ob1 = oW1 + H * DIN, oW2 = ob1 + H, ob2 = oW2 + H * H,
            ow3 = ob2 + H, ob3 = ow3 + H;
  for (int i = tid; i < H * DIN; i += NT) W1[i] = bf2f(wbf[oW1 + i]);
  for (int i = tid; i < H * H; i += NT) W2[i] = bf2f(wbf[oW2 + i]);
  if (tid < H) {
    b1[tid] = bf2f(wbf[ob1 + tid]);
    b2[tid] = bf2f(wbf[ob2 + tid]);
    w3[tid] = bf2f(wbf[ow3 + tid]);
  }
  if (tid == 0) {
    b3s = bf2f(wbf[ob3]);
    lsum = 0.f;
  }
  __syncthreads();
  float gW2[4] = {0, 0, 0, 0}, gW1[3] = {0, 0, 0}, gb1 = 0, gb2 = 0, gw3 = 0, gb3 = 0;
  const long long ntiles = (n + T_TILE - 1) / T_TILE;
  for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const long long base = tile * T_TILE;
    // 1. inputs of the tile's records
    if (tid < T_TILE) {
      const long long i = base + tid;
      float *x = X + tid * DIN;
      if (i < n) {
        const uint64_t r = rec[i];
        const int sym = (int)(r & 0xffff);
        const int ar = (int)((r >> 16) & 15);
        const int bits = (int)((r >> 20) & 31);
        const int bucket = (int)((r >> 25) & 15);
        for (int k = 0; k < EMB; k++) x[k] = bf2f(wbf[sym * EMB + k]);
        x[EMB] = ar / 8.0f;
        for (int j = 0; j < 5; j++) x[EMB + 1 + j] = (float)((bits >> j) & 1);
        x[EMB + 6] = bucket / 15.0f;
        x[EMB + 7] = 0.f;
        Y[tid] = (float)((r >> 32) & 1);
        SYM[tid] = sym;
      } else {
        for (int k = 0; k < DIN; k++) x[k] = 0.f;
        Y[tid] = -1.f;  // padding row
        SYM[tid] = 0;
      }
    }
    __syncthreads();
    // 2. H1 = relu(X W1^T + b1): thread -> record tid/4, hidden units 8(tid%4)..+8
    {
      const int t = tid >> 2, j0 = (tid & 3) * 8;
      for (int j = j0; j < j0 + 8; j++) {
        float acc = b1[j];
        for (int k = 0; k < DIN; k++) acc += W1[j * DIN + k] * X[t * DIN + k];
        H1[t * H + j] = acc > 0.f ? acc : 0.f;
      }
    }
    __syncthreads();
    // 3. H2 = relu(H1 W2^T + b2)
    {
      const int t = tid >> 2, j0 = (tid & 3) * 8;
      for (int j = j0; j < j0 + 8; j++) {
        float acc = b2[j];
        for (int k = 0; k < H; k++) acc += W2[j * H + k] * H1[t * H + k];
        H2[t * H + j] = acc > 0.f ? acc : 0.f;
      }
    }
    __syncthreads();
    // 4. output, loss, dL/dz
    if (tid < T_TILE) {
      float z = b3s;
      for (int k = 0; k < H; k++) z += w3[k] * H2[tid * H + k];
      const float y = Y[tid];
      const float p = 1.f / (1.f + expf(-z));
      float dz = 0.f;
      if (y >= 0.f) {
        const float sp = z > 0.f ? z + log1pf(expf(-z)) : log1pf(expf(z));
        atomicAdd(&lsum, sp - y * z);
        dz = (p - y) * scale;
        if (probs) probs[base + tid] = p;
      }
      DZ[tid] = dz;
    }
    __syncthreads();
    if (!want_grad) continue;
    // 5. dH2 = dz w3 (through relu)
    {
      const int t = tid >> 2, j0 = (tid & 3) * 8;
      for (int j = j0; j < j0 + 8; j++)
        D[t * H + j] = H2[t * H + j] > 0.f ? DZ[t] * w3[j] : 0.f;
    }
    __syncthreads();
    // 6. w3, b2, b3 gradients; 7. W2 gradient (4 entries per thread)
    if (tid < H) {
      float a = 0.f, b = 0.f;
      for (int t = 0; t < T_TILE; t++) {
        a += DZ[t] * H2[t * H + tid];
        b += D[t * H + tid];
      }
      gw3 += a;
      gb2 += b;
    }
    if (tid == 0) {
      float a = 0.f;
      for (int t = 0; t < T_TILE; t++) a += DZ[t];
      gb3 += a;
    }
    for (int e = 0; e < 4; e++) {
      const int idx = tid * 4 + e;  // 0..1023
      const int j = idx / H, k = idx % H;
      float a = 0.f;
      for (int t = 0; t < T_TILE; t++) a += D[t * H + j] * H1[t * H + k];
      gW2[e] += a;
    }
    __syncthreads();
    // 8. dH1 = dH2 W2 (through relu), written over H2
    {
      const int t = tid >> 2, k0 = (tid & 3) * 8;
      for (int k = k0; k < k0 + 8; k++) {
        float acc = 0.f;
        for (int j = 0; j < H; j++) acc += D[t * H + j] * W2[j * H + k];
        H2[t * H + k] = H1[t * H + k] > 0.f ? acc : 0.f;
      }
    }
    __syncthreads();
    // 9. b1 and W1 gradients (3 entries per thread: 768 = 256 x 3)
    if (tid < H) {
      float a = 0.f;
      for (int t = 0; t < T_TILE; t++) a += H2[t * H + tid];
      gb1 += a;
    }
    for (int e = 0; e < 3; e++) {
      const int idx = tid * 3 + e;  // 0..767
      const int j = idx / DIN, m = idx % DIN;
      float a = 0.f;
      for (int t = 0; t < T_TILE; t++) a += H2[t * H + j] * X[t * DIN + m];
      gW1[e] += a;
    }
    // 10. embedding gradient: dX[:, :16] = dH1 W1[:, :16], scattered by symbol
    for (int e = 0; e < 4; e++) {
      const int idx = tid * 4 + e;  // 0..1023 = 64 records x 16
      const int t = idx / EMB, m = idx % EMB;
      if (Y[t] < 0.f) continue;
      float a = 0.f;
      for (int j = 0; j < H; j++) a += H2[t * H + j] * W1[j * DIN + m];
      atomicAdd(&grad[SYM[t] * EMB + m], a);
    }
    __syncthreads();
  }
  if (want_grad) {
    for (int e = 0; e < 4; e++) atomicAdd(&grad[oW2 + tid * 4 + e], gW2[e]);
    for (int e = 0; e < 3; e++) atomicAdd(&grad[oW1 + tid * 3 + e], gW1[e]);
    if (tid < H) {
      atomicAdd(&grad[ob1 + tid], gb1);
      atomicAdd(&grad[ob2 + tid], gb2);
      atomicAdd(&grad[ow3 + tid], gw3);
    }
    if (tid == 0) atomicAdd(&grad[ob3], gb3);
  }
  __syncthreads();
  if (tid == 0) atomicAdd(loss, lsum);
}

// Adam step on float32 master weights; writes the bfloat16 copy and clears
// the gradient for the next step.
__global__ void k_adam(float *w, float *g, float *m, float *v, uint16_t *wbf, int P, float lr,
                       float beta1, float beta2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  const float gi = g[i];
  const float mi = beta1 * m[i] + (1.f - beta1) * gi;
  const float vi = beta2 * v[i] + (1.f - beta2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w[i] = wi;
  wbf[i] = f2bf(wi);
  g[i] = 0.f;
}

// One record per possible input (sym, bits, bucket), in table order.
__global__ void k_enum_inputs(int n_sym, const int32_t *arity, uint64_t *rec) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_sym * 512) return;
  const int sym = i >> 9, bits = (i >> 4) & 31, bucket = i & 15;
  rec[i] = (uint64_t)sym | ((uint64_t)(arity[sym] & 15) << 16) | ((uint64_t)bits << 20) |
           ((uint64_t)bucket << 25);
}

// Pack the keep decisions: bit i of word i/32 is p[i] >= threshold.
__global__ void k_pack_table(const float *p, int n, float threshold, uint32_t *words) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w * 32 >= n) return;
  uint32_t v = 0;
  for (int b = 0; b < 32; b++) {
    const int i = w * 32 + b;
    if (i < n && p[i] >= threshold) v |= 1u << b;
  }
  words[w] = v;
}

}  // namespace

int64_t trs_mlp_param_count(int32_t n_sym) {
  if (n_sym <= 0 || n_sym > TRS_MLP_MAX_SYM) return -1;
  return (int64_t)EMB * n_sym + H * DIN + H + H * H + H + H + 1;
}

hipError_t trs_mlp_build_table(const uint16_t *d_params, int n_sym, const int32_t *d_arity,
                               float threshold, float *d_probs, uint64_t *d_rec, float *d_loss,
                               uint32_t *d_words, hipStream_t s) {
  const int n = n_sym * 512;
  hipLaunchKernelGGL(k_enum_inputs, dim3((n + 255) / 256), dim3(256), 0, s, n_sym, d_arity,
                     d_rec);
  const int tiles = (n + T_TILE - 1) / T_TILE;
  hipLaunchKernelGGL(k_mlp_grad, dim3(tiles < 1024 ? tiles : 1024), dim3(NT), 0, s, d_params,
                     n_sym, (const uint64_t *)d_rec, (long long)n, 1.0f, (float *)nullptr, d_loss,
                     d_probs, 0);
  hipLaunchKernelGGL(k_pack_table, dim3((n / 32 + 255) / 256), dim3(256), 0, s,
                     (const float *)d_probs, n, threshold, d_words);
  return hipGetLastError();
}

#define CK(x)                \
  do {                       \
    if ((x) != hipSuccess) { \
      st = TRS_E_HIP;        \
      goto out;              \
    }                        \
  } while (0)

static bool records_valid(int32_t n_sym, int64_t n, const uint64_t *records) {
  for (int64_t i = 0; i < n; i++)
    if ((int64_t)(records[i] & 0xffff) >= n_sym) return false;
  return true;
}

extern "C" trs_status trs_mlp_eval(int32_t device, int32_t n_sym, const uint16_t *params_bf16,
                                   int64_t n, const uint64_t *records, double *loss_out,
                                   float *grads_out, float *probs_out) {
  const int64_t P = trs_mlp_param_count(n_sym);
  if (P < 0 || !params_bf16 || n <= 0 || !records || !loss_out) return TRS_E_ARG;
  if (!records_valid(n_sym, n, records)) return TRS_E_ARG;
  trs_status st = TRS_OK;
  uint16_t *dw = nullptr;
  uint64_t *dr = nullptr;
  float *dg = nullptr, *dl = nullptr, *dp = nullptr;
  float hl = 0.f;
  CK(hipSetDevice(device));
  CK(hipMalloc(&dw, P * 2));
  CK(hipMalloc(&dr, n * 8));
  CK(hipMalloc(&dg, P * 4));
  CK(hipMalloc(&dl, 4));
  if (probs_out) CK(hipMalloc(&dp, n * 4));
  CK(hipMemcpy(dw, params_bf16, P * 2, hipMemcpyHostToDevice));
  CK(hipMemcpy(dr, records, n * 8, hipMemcpyHostToDevice));
  CK(hipMemset(dg, 0, P * 4));
  CK(hipMemset(dl, 0, 4));
  {
    const int64_t tiles = (n + T_TILE - 1) / T_TILE;
    const int G = (int)(tiles < 1024 ? tiles : 1024);
    hipLaunchKernelGGL(k_mlp_grad, dim3(G), dim3(NT), 0, 0, dw, n_sym, dr, (long long)n,
                       1.0f / (float)n, dg, dl, dp, grads_out ? 1 : 0);
    CK(hipGetLastError());
  }
  CK(hipDeviceSynchronize());
  CK(hipMemcpy(&hl, dl, 4, hipMemcpyDeviceToHost));
  *loss_out = (double)hl / (double)n;
  if (grads_out) CK(hipMemcpy(grads_out, dg, P * 4, hipMemcpyDeviceToHost));
  if (probs_out) CK(hipMemcpy(probs_out, dp, n * 4, hipMemcpyDeviceToHost));
out:
  (void)hipFree(dw);
  (void)hipFree(dr);
  (void)hipFree(dg);
  (void)hipFree(dl);
  (void)hipFree(dp);
  return st;
}

// ------------------------------------------------------------------------
// trs_mlp_eval_noalloc: trs_mlp_eval with every device buffer (parameters,
// records, gradient and loss accumulators, probabilities) in one static
// device array, so the call allocates nothing.  Each device holds its own
// copy of the array until the process ends; its address on a device is taken
// once, with that device current, by hipGetSymbolAddress, and only that
// address is handed to kernels and copies (the array's name is a host-side
// stand-in in host code).  Calls on one device share the array: calls that
// overlap in time on one device race.
#define NOALLOC_P_MAX 6144  // >= trs_mlp_param_count(TRS_MLP_MAX_SYM) = 5985
constexpr size_t NA_OFF_W = 0;                                      // bfloat16 params
constexpr size_t NA_OFF_G = NA_OFF_W + NOALLOC_P_MAX * 2;           // float gradient
constexpr size_t NA_OFF_L = NA_OFF_G + NOALLOC_P_MAX * 4;           // float loss (256 B)
constexpr size_t NA_OFF_R = NA_OFF_L + 256;                         // uint64 records
constexpr size_t NA_OFF_P = NA_OFF_R + (size_t)TRS_MLP_NOALLOC_MAX_RECORDS * 8;  // float p
constexpr size_t NA_BYTES = NA_OFF_P + (size_t)TRS_MLP_NOALLOC_MAX_RECORDS * 4;
static_assert(NA_OFF_G % 256 == 0 && NA_OFF_L % 256 == 0 && NA_OFF_R % 256 == 0 &&
                  NA_OFF_P % 256 == 0,
              "scratch sections stay 256-byte aligned");

static __device__ __align__(256) unsigned char scratch[NA_BYTES];

namespace {

#define NA_MAX_DEVICES 64
std::mutex g_na_mutex;
void *g_na_ptr[NA_MAX_DEVICES];  // device address of `scratch` per device (null: not yet)

// The device address of this device's copy of `scratch` (the caller has made
// `device` current); null on failure.
void *noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_na_mutex);
  if (!g_na_ptr[device]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    g_na_ptr[device] = ptr;
  }
  return g_na_ptr[device];
}

// Clears n floats (the accumulators must start at zero; a kernel rather than
// a memset node).
__global__ void k_zero_f32(float *p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

}  // namespace

extern "C" trs_status trs_mlp_eval_noalloc(int32_t device, int32_t n_sym,
                                           const uint16_t *params_bf16, int64_t n,
                                           const uint64_t *records, double *loss_out,
                                           float *grads_out, float *probs_out) {
  const int64_t P = trs_mlp_param_count(n_sym);
  if (P < 0 || !params_bf16 || n <= 0 || !records || !loss_out) return TRS_E_ARG;
  if (n > TRS_MLP_NOALLOC_MAX_RECORDS || P > NOALLOC_P_MAX) return TRS_E_LIMIT;
  if (device < 0 || device >= NA_MAX_DEVICES) return TRS_E_ARG;
  if (!records_valid(n_sym, n, records)) return TRS_E_ARG;
  trs_status st = TRS_OK;
  float hl = 0.f;
  char *base = nullptr;
  uint16_t *dw;
  float *dg, *dl, *dp;
  uint64_t *dr;
  CK(hipSetDevice(device));
  base = (char *)noalloc_scratch(device);
  if (!base) return TRS_E_HIP;
  dw = (uint16_t *)(base + NA_OFF_W);
  dg = (float *)(base + NA_OFF_G);
  dl = (float *)(base + NA_OFF_L);
  dr = (uint64_t *)(base + NA_OFF_R);
  dp = probs_out ? (float *)(base + NA_OFF_P) : nullptr;
  CK(hipMemcpy(dw, params_bf16, P * 2, hipMemcpyHostToDevice));
  CK(hipMemcpy(dr, records, n * 8, hipMemcpyHostToDevice));
  // the previous call's gradient and loss are still there
  hipLaunchKernelGGL(k_zero_f32, dim3((unsigned)((P + 1 + 255) / 256)), dim3(256), 0, 0, dg,
                     (int)P);
  hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(64), 0, 0, dl, 1);
  CK(hipGetLastError());
  {
    const int64_t tiles = (n + T_TILE - 1) / T_TILE;
    const int G = (int)(tiles < 1024 ? tiles : 1024);
    hipLaunchKernelGGL(k_mlp_grad, dim3(G), dim3(NT), 0, 0, (const uint16_t *)dw, n_sym,
                       (const uint64_t *)dr, (long long)n, 1.0f / (float)n, dg, dl, dp,
                       grads_out ? 1 : 0);
    CK(hipGetLastError());
  }
  CK(hipDeviceSynchronize());
  CK(hipMemcpy(&hl, dl, 4, hipMemcpyDeviceToHost));
  *loss_out = (double)hl / (double)n;
  if (grads_out) CK(hipMemcpy(grads_out, dg, P * 4, hipMemcpyDeviceToHost));
  if (probs_out) CK(hipMemcpy(probs_out, dp, n * 4, hipMemcpyDeviceToHost));
out:
  return st;
}

extern "C" trs_status trs_mlp_train(int32_t device, int32_t n_sym, int64_t n,
                                    const uint64_t *records, const trs_train_opts *opts,
                                    const uint16_t *init_bf16, uint16_t *params_out,
                                    trs_train_result *res) {
  const int64_t P = trs_mlp_param_count(n_sym);
  if (P < 0 || n < 2 || !records || !opts || !init_bf16 || !params_out) return TRS_E_ARG;
  if (opts->epochs < 1 || opts->epochs > 64 || opts->batch < T_TILE || !(opts->lr > 0.f) ||
      !(opts->val_frac >= 0.f) || !(opts->val_frac < 1.f))
    return TRS_E_ARG;
  if (!records_valid(n_sym, n, records)) return TRS_E_ARG;
  const int64_t nval = (int64_t)(opts->val_frac * (double)n);
  const int64_t ntrain = n - nval;
  if (ntrain < 1) return TRS_E_ARG;
  trs_status st = TRS_OK;
  trs_train_result r;
  std::memset(&r, 0, sizeof(r));
  uint16_t *dwb = nullptr;
  uint64_t *dr = nullptr;
  float *dw = nullptr, *dg = nullptr, *dm = nullptr, *dv = nullptr, *dl = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  std::vector<float> w0(P);
  for (int64_t i = 0; i < P; i++) {
    const uint32_t u = (uint32_t)init_bf16[i] << 16;
    std::memcpy(&w0[i], &u, 4);
  }
  CK(hipSetDevice(device));
  CK(hipMalloc(&dwb, P * 2));
  CK(hipMalloc(&dr, n * 8));
  CK(hipMalloc(&dw, P * 4));
  CK(hipMalloc(&dg, P * 4));
  CK(hipMalloc(&dm, P * 4));
  CK(hipMalloc(&dv, P * 4));
  CK(hipMalloc(&dl, 4));
  CK(hipMemcpy(dwb, init_bf16, P * 2, hipMemcpyHostToDevice));
  CK(hipMemcpy(dw, w0.data(), P * 4, hipMemcpyHostToDevice));
  CK(hipMemcpy(dr, records, n * 8, hipMemcpyHostToDevice));
  CK(hipMemset(dg, 0, P * 4));
  CK(hipMemset(dm, 0, P * 4));
  CK(hipMemset(dv, 0, P * 4));
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  CK(hipEventRecord(e0, 0));
  {
    const int B = opts->batch;
    const float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
    double b1t = 1.0, b2t = 1.0;
    for (int ep = 0; ep < opts->epochs; ep++) {
      CK(hipMemset(dl, 0, 4));
      for (int64_t off = 0; off < ntrain; off += B) {
        const int64_t nb = ntrain - off < B ? ntrain - off : B;
        const int64_t tiles = (nb + T_TILE - 1) / T_TILE;
        const int G = (int)(tiles < 256 ? tiles : 256);
        hipLaunchKernelGGL(k_mlp_grad, dim3(G), dim3(NT), 0, 0, dwb, n_sym, dr + off,
                           (long long)nb, 1.0f / (float)nb, dg, dl, (float *)nullptr, 1);
        b1t *= beta1;
        b2t *= beta2;
        hipLaunchKernelGGL(k_adam, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, 0, dw, dg,
                           dm, dv, dwb, (int)P, opts->lr, beta1, beta2, eps, (float)(1.0 - b1t),
                           (float)(1.0 - b2t));
      }
      CK(hipGetLastError());
      float hl = 0.f;
      CK(hipMemcpy(&hl, dl, 4, hipMemcpyDeviceToHost));
      r.train_loss[ep] = hl / (float)ntrain;
      if (nval > 0) {
        CK(hipMemset(dl, 0, 4));
        const int64_t tiles = (nval + T_TILE - 1) / T_TILE;
        const int G = (int)(tiles < 1024 ? tiles : 1024);
        hipLaunchKernelGGL(k_mlp_grad, dim3(G), dim3(NT), 0, 0, dwb, n_sym, dr + ntrain,
                           (long long)nval, 1.0f, (float *)nullptr, dl, (float *)nullptr, 0);
        CK(hipGetLastError());
        CK(hipMemcpy(&hl, dl, 4, hipMemcpyDeviceToHost));
        r.val_loss[ep] = hl / (float)nval;
      }
      r.epochs_run = ep + 1;
    }
  }
  CK(hipEventRecord(e1, 0));
  CK(hipEventSynchronize(e1));
  {
    float ms = 0.f;
    CK(hipEventElapsedTime(&ms, e0, e1));
    r.device_ms = ms;
  }
  CK(hipMemcpy(params_out, dwb, P * 2, hipMemcpyDeviceToHost));
  if (res) *res = r;
out:
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(dwb);
  (void)hipFree(dr);
  (void)hipFree(dw);
  (void)hipFree(dg);
  (void)hipFree(dm);
  (void)hipFree(dv);
  (void)hipFree(dl);
  return st;
}

extern "C" trs_status trs_mlp_table(int32_t device, int32_t n_sym, const int32_t *arity,
                                    const uint16_t *params_bf16, float threshold,
                                    float *probs_out, uint32_t *words_out) {
  const int64_t P = trs_mlp_param_count(n_sym);
  if (P < 0 || !arity || !params_bf16) return TRS_E_ARG;
  for (int i = 0; i < n_sym; i++)
    if (arity[i] < 0 || arity[i] > 15) return TRS_E_ARG;
  trs_status st = TRS_OK;
  const int n = n_sym * 512;
  uint16_t *dw = nullptr;
  int32_t *da = nullptr;
  float *dp = nullptr, *dl = nullptr;
  uint64_t *dr = nullptr;
  uint32_t *dt = nullptr;
  CK(hipSetDevice(device));
  CK(hipMalloc(&dw, P * 2));
  CK(hipMalloc(&da, n_sym * 4));
  CK(hipMalloc(&dp, (size_t)n * 4));
  CK(hipMalloc(&dl, 4));
  CK(hipMalloc(&dr, (size_t)n * 8));
  CK(hipMalloc(&dt, (size_t)n / 8));
  CK(hipMemcpy(dw, params_bf16, P * 2, hipMemcpyHostToDevice));
  CK(hipMemcpy(da, arity, n_sym * 4, hipMemcpyHostToDevice));
  CK(hipMemset(dl, 0, 4));
  CK(trs_mlp_build_table(dw, n_sym, da, threshold, dp, dr, dl, dt, 0));
  CK(hipDeviceSynchronize());
  if (probs_out) CK(hipMemcpy(probs_out, dp, (size_t)n * 4, hipMemcpyDeviceToHost));
  if (words_out) CK(hipMemcpy(words_out, dt, (size_t)n / 8, hipMemcpyDeviceToHost));
out:
  (void)hipFree(dw);
  (void)hipFree(da);
  (void)hipFree(dp);
  (void)hipFree(dl);
  (void)hipFree(dr);
  (void)hipFree(dt);
  return st;
}
