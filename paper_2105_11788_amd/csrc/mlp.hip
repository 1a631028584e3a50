// The splitter-scoring network: y = w3 . relu(W2 relu(W1 x + b1) + b2) + b3,
// hidden width 64, F inputs.  fp32 master parameters; the forward pass uses
// bf16 copies of all parameters and of the input (round to nearest even) and
// accumulates in fp32 on the vector ALUs (a few kFLOP per row: far too small
// for matrix cores to matter).  Training: mean squared error, gradients with
// respect to the bf16 copies, Adam on the fp32 masters.
//
// Kernels
//   k_mlp_forward   one wave per row; lane j is hidden unit j; weights staged
//                   in LDS as fp32, W1 and W2 transposed so that lanes read
//                   consecutive words.
//   k_mlp_backward  same row mapping; each wave keeps lane j's slice of the
//                   weight gradients in registers over its rows, then the
//                   workgroup reduces through LDS (waves in a fixed order)
//                   and stores its partial sums in its own row of a
//                   partials buffer.
//   k_mlp_sum       sums the workgroups' partials of each parameter in
//                   workgroup order: no floating-point atomics, so a training
//                   step is bitwise reproducible.
//   k_mlp_adam      elementwise Adam step, refreshes the bf16 copy.
#include <cmath>
#include <new>
#include <vector>

#include "internal.h"
#include "mlp_dev.h"

struct bisim_mlp {
  int F = 0;
  int64_t P = 0;
  float* master = nullptr;   // device fp32 [P]
  uint16_t* wbf = nullptr;   // device bf16 [P]
  float* m = nullptr;        // Adam moments
  float* v = nullptr;
  float* grad = nullptr;     // device fp32 [P]
  float* loss = nullptr;     // device fp32 [1]
  float* part = nullptr;     // device fp32 [workgroups][P + 2]: partial sums (+ b3, loss)
  int64_t step = 0;
};

namespace bisim {
namespace {
constexpr int kMT = 256;  // 4 waves per workgroup

__global__ void __launch_bounds__(kMT) k_mlp_forward(const uint16_t* __restrict__ w, int F,
                                                      const float* __restrict__ x, int64_t rows,
                                                      float* __restrict__ y) {
  extern __shared__ float sw[];
  MlpLds L = mlp_lds_layout(sw, F);
  mlp_stage(L, w, F);
  __syncthreads();
  const int64_t wave = ((int64_t)blockIdx.x * kMT + threadIdx.x) / kWave;
  const int64_t nwaves = (int64_t)gridDim.x * kMT / kWave;
  for (int64_t r = wave; r < rows; r += nwaves) {
    float z1, z2;
    const float out = mlp_row_forward(L, F, x + r * F, &z1, &z2);
    if (lane() == 0) y[r] = out;
  }
}

// the same with bf16 inputs (raw IEEE bf16 bits): exact in fp32, and already
// at the precision the forward pass rounds its inputs to
__global__ void __launch_bounds__(kMT) k_mlp_forward_bf16(const uint16_t* __restrict__ w, int F,
                                                           const uint16_t* __restrict__ x,
                                                           int64_t rows, float* __restrict__ y) {
  extern __shared__ float sw[];
  MlpLds L = mlp_lds_layout(sw, F);
  mlp_stage(L, w, F);
  __syncthreads();
  const int64_t wave = ((int64_t)blockIdx.x * kMT + threadIdx.x) / kWave;
  const int64_t nwaves = (int64_t)gridDim.x * kMT / kWave;
  const int j = (int)lane();
  for (int64_t r = wave; r < rows; r += nwaves) {
    const float xl = j < F ? __uint_as_float((uint32_t)x[r * F + j] << 16) : 0.f;
    float z1, z2;
    const float out = mlp_forward_lanes(L, F, xl, &z1, &z2);
    if (lane() == 0) y[r] = out;
  }
}

__global__ void __launch_bounds__(kMT) k_mlp_backward(const uint16_t* __restrict__ w, int F,
                                                       const float* __restrict__ x,
                                                       const float* __restrict__ t, int64_t rows,
                                                       float* __restrict__ part, int64_t P) {
  extern __shared__ float sw[];
  MlpLds L = mlp_lds_layout(sw, F);
  float* red = L.end;  // [kMT/64 waves][64 lanes] partial sums, one parameter row at a time
  mlp_stage(L, w, F);
  __syncthreads();
  const int j = (int)lane();
  const int wv = threadIdx.x / kWave;
  const int64_t wave = ((int64_t)blockIdx.x * kMT + threadIdx.x) / kWave;
  const int64_t nwaves = (int64_t)gridDim.x * kMT / kWave;
  const float inv = 2.0f / (float)rows;
  // lane j accumulates: gW2[j][0..63] (row j), gW1[j][0..F), gb1[j], gb2[j], gw3[j]; gb3, loss
  float gW2[kMlpH];
  float gW1[kMlpMaxF];
#pragma unroll
  for (int i = 0; i < kMlpH; ++i) gW2[i] = 0.f;
#pragma unroll
  for (int i = 0; i < kMlpMaxF; ++i) gW1[i] = 0.f;
  float gb1 = 0.f, gb2 = 0.f, gw3 = 0.f, gb3 = 0.f, lsum = 0.f;
  for (int64_t r = wave; r < rows; r += nwaves) {
    const float* xr = x + r * F;
    float z1, z2;
    const float yv = mlp_row_forward(L, F, xr, &z1, &z2);
    const float h1 = fmaxf(z1, 0.f), h2 = fmaxf(z2, 0.f);
    const float diff = yv - t[r];
    const float dy = inv * diff;
    lsum += diff * diff;
    gb3 += dy;
    gw3 += dy * h2;
    const float dz2 = (z2 > 0.f) ? dy * L.w3[j] : 0.f;
    gb2 += dz2;
    // gW2[j][i] += dz2_j * h1_i ; dh1_j = sum_i dz2_i * W2[i][j]
    float dh1 = 0.f;
#pragma unroll
    for (int i = 0; i < kMlpH; ++i) {
      const float h1i = __shfl(h1, i, kWave);
      const float dz2i = __shfl(dz2, i, kWave);
      gW2[i] += dz2 * h1i;
      dh1 += dz2i * L.W2[i * kMlpH + j];
    }
    const float dz1 = (z1 > 0.f) ? dh1 : 0.f;
    gb1 += dz1;
#pragma unroll
    for (int f = 0; f < kMlpMaxF; ++f)
      if (f < F) gW1[f] += dz1 * bf16_rne(xr[f]);
  }
  // workgroup reduction through LDS (waves summed in order), one store per
  // parameter into this workgroup's row of the partials
  float* mine = part + (int64_t)blockIdx.x * (P + 2);
  auto reduce_store = [&](float v, int64_t idx) {
    red[wv * kWave + j] = v;
    __syncthreads();
    if (wv == 0) {
      float s = 0.f;
      for (int q = 0; q < kMT / kWave; ++q) s += red[q * kWave + j];
      mine[idx] = s;
    }
    __syncthreads();
  };
  const MlpOffsets o = mlp_offsets(F);
  for (int i = 0; i < kMlpH; ++i) reduce_store(gW2[i], o.W2 + j * kMlpH + i);
  for (int f = 0; f < F; ++f) reduce_store(gW1[f], o.W1 + j * F + f);
  reduce_store(gb1, o.b1 + j);
  reduce_store(gb2, o.b2 + j);
  reduce_store(gw3, o.w3 + j);
  // scalars: every lane of a wave holds the same dy sum (b3) and the same
  // squared errors (the row's output is the wave's); lane 0's, then the
  // waves in order
  if (j == 0) {
    red[wv] = gb3;
    red[kMT / kWave + wv] = lsum;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float sb = 0.f, sl = 0.f;
    for (int q = 0; q < kMT / kWave; ++q) {
      sb += red[q];
      sl += red[kMT / kWave + q];
    }
    mine[o.b3] = sb;
    mine[P + 1] = sl / (float)rows;
  }
}

// sum of the workgroups' partials, in workgroup order; index P + 1 is the loss
__global__ void k_mlp_sum(const float* __restrict__ part, int nblk, int64_t P,
                          float* __restrict__ grad, float* __restrict__ loss) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= P + 1;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i == P) continue;
    float s = 0.f;
    for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * (P + 2) + i];
    if (i == P + 1) *loss = s;
    else grad[i] = s;
  }
}

__global__ void k_mlp_adam(float* __restrict__ w, uint16_t* __restrict__ wbf,
                           float* __restrict__ m, float* __restrict__ v,
                           const float* __restrict__ g, int64_t P, float lr, float c1, float c2) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    wbf[i] = bf16_bits(wi);
  }
}

__global__ void k_to_bf16(const float* __restrict__ w, uint16_t* __restrict__ wbf, int64_t P) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P;
       i += (int64_t)gridDim.x * blockDim.x)
    wbf[i] = bf16_bits(w[i]);
}

// He-normal initialisation from splitmix64 + Box-Muller (host side)
uint64_t splitmix64(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
double normal(uint64_t& s) {
  const double u1 = ((splitmix64(s) >> 11) + 1.0) * (1.0 / 9007199254740993.0);
  const double u2 = (splitmix64(s) >> 11) * (1.0 / 9007199254740992.0);
  return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
}

size_t fwd_lds(int F) { return mlp_lds_floats(F) * sizeof(float); }
size_t bwd_lds(int F) { return (mlp_lds_floats(F) + (kMT / kWave) * kWave) * sizeof(float); }

constexpr int kMaxGridRows = 1024;
unsigned grid_rows(int64_t rows) {
  int64_t waves = (rows + 0) / 1;
  int64_t g = (waves + (kMT / kWave) - 1) / (kMT / kWave);
  if (g > kMaxGridRows) g = kMaxGridRows;
  if (g < 1) g = 1;
  return (unsigned)g;
}
}  // namespace

bisim_status mlp_forward_dev(const bisim_mlp* w, const float* x, int64_t rows, float* y,
                             hipStream_t s) {
  if (rows <= 0) return BISIM_OK;
  hipLaunchKernelGGL(k_mlp_forward, dim3(grid_rows(rows)), dim3(kMT), fwd_lds(w->F), s, w->wbf,
                     w->F, x, rows, y);
  BISIM_TRY_HIP(hipGetLastError());
  return BISIM_OK;
}
const uint16_t* mlp_weights_bf16(const bisim_mlp* w) { return w->wbf; }
int mlp_features(const bisim_mlp* w) { return w->F; }
}  // namespace bisim

using namespace bisim;

extern "C" {

int64_t mlp_num_params(int32_t in_features) {
  if (in_features < 1 || in_features > kMlpMaxF) return -1;
  return mlp_offsets(in_features).total;
}

bisim_status mlp_create(int32_t in_features, const float* init_fp32, uint64_t seed,
                        bisim_mlp** out) {
  if (!out || in_features < 1 || in_features > kMlpMaxF) {
    set_error("mlp_create: need 1 <= in_features <= %d and an output pointer", kMlpMaxF);
    return BISIM_E_INVALID;
  }
  *out = nullptr;
  bisim_mlp* w = new (std::nothrow) bisim_mlp;
  if (!w) return BISIM_E_NOMEM;
  w->F = in_features;
  w->P = mlp_offsets(in_features).total;
  std::vector<float> h((size_t)w->P, 0.f);
  if (init_fp32) {
    for (int64_t i = 0; i < w->P; ++i) h[i] = init_fp32[i];
  } else {
    const MlpOffsets o = mlp_offsets(in_features);
    uint64_t s = seed;
    for (int i = 0; i < kMlpH * in_features; ++i)
      h[o.W1 + i] = (float)(normal(s) * std::sqrt(2.0 / in_features));
    for (int i = 0; i < kMlpH * kMlpH; ++i) h[o.W2 + i] = (float)(normal(s) * std::sqrt(2.0 / kMlpH));
    for (int i = 0; i < kMlpH; ++i) h[o.w3 + i] = (float)(normal(s) * std::sqrt(1.0 / kMlpH));
  }
  hipError_t e = hipMalloc((void**)&w->master, 4 * w->P);
  if (e == hipSuccess) e = hipMalloc((void**)&w->wbf, 2 * w->P);
  if (e == hipSuccess) e = hipMalloc((void**)&w->m, 4 * w->P);
  if (e == hipSuccess) e = hipMalloc((void**)&w->v, 4 * w->P);
  if (e == hipSuccess) e = hipMalloc((void**)&w->grad, 4 * w->P);
  if (e == hipSuccess) e = hipMalloc((void**)&w->loss, 4);
  if (e == hipSuccess) e = hipMalloc((void**)&w->part, 4 * (size_t)kMaxGridRows * (w->P + 2));
  if (e == hipSuccess) e = hipMemcpy(w->master, h.data(), 4 * w->P, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(w->m, 0, 4 * w->P);
  if (e == hipSuccess) e = hipMemset(w->v, 0, 4 * w->P);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_to_bf16, dim3(16), dim3(256), 0, nullptr, w->master, w->wbf, w->P);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    set_error("mlp_create: %s", hipGetErrorString(e));
    mlp_free(w);
    return BISIM_E_DEVICE;
  }
  *out = w;
  return BISIM_OK;
}

void mlp_free(bisim_mlp* w) {
  if (!w) return;
  (void)hipDeviceSynchronize();
  void* p[] = {w->master, w->wbf, w->m, w->v, w->grad, w->loss, w->part};
  for (void* q : p)
    if (q) (void)hipFree(q);
  delete w;
}

bisim_status mlp_get_params(const bisim_mlp* w, float* host_fp32) {
  if (!w || !host_fp32) {
    set_error("mlp_get_params: NULL argument");
    return BISIM_E_INVALID;
  }
  BISIM_TRY_HIP(hipDeviceSynchronize());
  BISIM_TRY_HIP(hipMemcpy(host_fp32, w->master, 4 * w->P, hipMemcpyDeviceToHost));
  return BISIM_OK;
}

bisim_status mlp_forward(const bisim_mlp* w, const float* x, int64_t rows, float* y,
                         void* hip_stream) {
  if (!w || rows < 0 || (rows > 0 && (!x || !y))) {
    set_error("mlp_forward: bad arguments");
    return BISIM_E_INVALID;
  }
  BISIM_TRY(mlp_forward_dev(w, x, rows, y, (hipStream_t)hip_stream));
  BISIM_TRY_HIP(hipStreamSynchronize((hipStream_t)hip_stream));
  return BISIM_OK;
}

bisim_status mlp_forward_bf16(const bisim_mlp* w, const void* x_bf16, int64_t rows, float* y,
                              void* hip_stream) {
  if (!w || rows < 0 || (rows > 0 && (!x_bf16 || !y))) {
    set_error("mlp_forward_bf16: bad arguments");
    return BISIM_E_INVALID;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  if (rows > 0) {
    hipLaunchKernelGGL(k_mlp_forward_bf16, dim3(grid_rows(rows)), dim3(kMT), fwd_lds(w->F), s,
                       w->wbf, w->F, (const uint16_t*)x_bf16, rows, y);
    BISIM_TRY_HIP(hipGetLastError());
  }
  BISIM_TRY_HIP(hipStreamSynchronize(s));
  return BISIM_OK;
}

bisim_status mlp_train_step(bisim_mlp* w, const float* x, const float* target, int64_t rows,
                            float lr, float* loss_out, float* grad_out, void* hip_stream) {
  if (!w || rows < 1 || !x || !target || !(lr >= 0.f)) {
    set_error("mlp_train_step: bad arguments");
    return BISIM_E_INVALID;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  const unsigned g = grid_rows(rows);
  hipLaunchKernelGGL(k_mlp_backward, dim3(g), dim3(kMT), bwd_lds(w->F), s, w->wbf, w->F, x,
                     target, rows, w->part, w->P);
  hipLaunchKernelGGL(k_mlp_sum, dim3(32), dim3(256), 0, s, w->part, (int)g, w->P, w->grad,
                     w->loss);
  BISIM_TRY_HIP(hipGetLastError());
  if (grad_out)
    BISIM_TRY_HIP(hipMemcpyAsync(grad_out, w->grad, 4 * w->P, hipMemcpyDeviceToDevice, s));
  if (lr > 0.f) {
    w->step += 1;
    const float c1 = 1.f - std::pow(0.9f, (float)w->step);
    const float c2 = 1.f - std::pow(0.999f, (float)w->step);
    hipLaunchKernelGGL(k_mlp_adam, dim3(32), dim3(256), 0, s, w->master, w->wbf, w->m, w->v,
                       w->grad, w->P, lr, c1, c2);
    BISIM_TRY_HIP(hipGetLastError());
  }
  float l = 0.f;
  BISIM_TRY_HIP(hipMemcpyAsync(&l, w->loss, 4, hipMemcpyDeviceToHost, s));
  BISIM_TRY_HIP(hipStreamSynchronize(s));
  if (loss_out) *loss_out = l;
  return BISIM_OK;
}

}  // extern "C"
