// Throughput of the instruction classes the event pass is built from, on one GPU: FP32 FMA, the
// v_exp_f32 / v_rsq_f32 transcendentals alone and mixed with FMAs, LDS atomics of each width, and
// global 32-bit float atomics.  These rates are the slot costs of the pass's
// roofline (an FMA is one VALU issue slot; a transcendental, measured here, two).
//
// Build: hipcc -O3 --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops
//        -o microbench microbench.hip       (paper_1502_07478_amd/build.py does this)
// Run:   ./microbench      (about one second; prints one line per probe)
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <vector>

#define CHECK(x)                                                                     \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess) {                                                          \
      printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__);          \
      exit(1);                                                                       \
    }                                                                                \
  } while (0)

namespace {

constexpr int kIt = 1024;   // dependent steps per chain
constexpr int kLdsIt = 256; // LDS operations per lane
constexpr int kLdsN = 8192; // LDS words of the atomic probes (16 wavefronts x 512-word windows)

// eight independent FMA chains per lane
__global__ void k_fma(float* out, float a, float b) {
  float x[8];
  for (int j = 0; j < 8; ++j) x[j] = threadIdx.x * 1e-3f + j;
  for (int i = 0; i < kIt; ++i) {
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = fmaf(x[j], a, b);
  }
  float s = 0;
  for (int j = 0; j < 8; ++j) s += x[j];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// eight independent chains of one transcendental
template <bool RSQ>
__global__ void k_trans(float* out) {
  float x[8];
  for (int j = 0; j < 8; ++j) x[j] = 1.0f + threadIdx.x * 1e-3f + j * 0.1f;
  for (int i = 0; i < kIt; ++i) {
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = RSQ ? __builtin_amdgcn_rsqf(x[j]) : __builtin_amdgcn_exp2f(-x[j]);
  }
  float s = 0;
  for (int j = 0; j < 8; ++j) s += x[j];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// per step: four exp2 chains and 8 NF FMAs on separate chains (do they overlap?)
template <int NF>
__global__ void k_mix(float* out, float a, float b) {
  float x[4], y[8];
  for (int j = 0; j < 4; ++j) x[j] = threadIdx.x * 1e-3f + j * 0.1f;
  for (int j = 0; j < 8; ++j) y[j] = threadIdx.x * 1e-3f + j;
  for (int i = 0; i < kIt; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) x[j] = __builtin_amdgcn_exp2f(-x[j]);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
#pragma unroll
      for (int j = 0; j < 8; ++j) y[j] = fmaf(y[j], a, b);
    }
  }
  float s = 0;
  for (int j = 0; j < 4; ++j) s += x[j];
  for (int j = 0; j < 8; ++j) s += y[j];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// LDS: every wavefront owns a 512-word window (16 wavefronts per workgroup), lanes walk it with
// unit stride, so accesses are conflict-free.  MODE 1 ds_add_f32, 2 ds_add_u32, 3 ds_add_u64,
// 4 ds_add_f64.
template <int MODE>
__global__ void __launch_bounds__(1024) k_lds(float* out) {
  __shared__ float lds[kLdsN];
  __shared__ double l64[kLdsN / 2];
  for (int i = threadIdx.x; i < kLdsN; i += blockDim.x) lds[i] = 0.0f;
  for (int i = threadIdx.x; i < kLdsN / 2; i += blockDim.x) l64[i] = 0.0;
  __syncthreads();
  const unsigned wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const unsigned win = wave * 512;
  for (int i = 0; i < kLdsIt; ++i) {
    const unsigned idx = win + ((lane + i * 64) & 511);
    if (MODE == 1) atomicAdd(&lds[idx], 1.0f);
    else if (MODE == 2) atomicAdd(reinterpret_cast<unsigned*>(&lds[idx]), 1u);
    else if (MODE == 3) atomicAdd(reinterpret_cast<unsigned long long*>(&l64[idx >> 1]), 1ull);
    else atomicAdd(&l64[idx >> 1], 1.0);
  }
  __syncthreads();
  float s = 0.0f;
  for (int i = threadIdx.x; i < kLdsN; i += blockDim.x) s += lds[i];
  for (int i = threadIdx.x; i < kLdsN / 2; i += blockDim.x) s += (float)l64[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// global float atomics without return: each wavefront adds to 64 consecutive words at a
// scattered base inside an array of n words
__global__ void k_gatomic(float* buf, unsigned n, int iters) {
  const unsigned gw = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const unsigned lane = threadIdx.x & 63;
  for (int i = 0; i < iters; ++i) {
    const unsigned base = ((gw * 7919u + i * 104729u) * 64u) % n;
    const unsigned idx = base + lane;
    if (idx < n) unsafeAtomicAdd(&buf[idx], 1.0f);
  }
}

template <typename F>
float time_ms(F f, int reps = 5) {
  hipEvent_t a, b;
  CHECK(hipEventCreate(&a));
  CHECK(hipEventCreate(&b));
  f();
  CHECK(hipGetLastError());
  CHECK(hipDeviceSynchronize());
  CHECK(hipEventRecord(a));
  for (int r = 0; r < reps; ++r) f();
  CHECK(hipEventRecord(b));
  CHECK(hipEventSynchronize(b));
  float ms = 0.0f;
  CHECK(hipEventElapsedTime(&ms, a, b));
  CHECK(hipEventDestroy(a));
  CHECK(hipEventDestroy(b));
  return ms / reps;
}

}  // namespace

int main() {
  hipDeviceProp_t p;
  CHECK(hipGetDeviceProperties(&p, 0));
  printf("device %s, %d CUs, %d kHz\n", p.gcnArchName, p.multiProcessorCount, p.clockRate);
  const int blocks = 256 * 32, threads = 256;
  float* out = nullptr;
  CHECK(hipMalloc(&out, sizeof(float) * (size_t)blocks * threads));
  const double lanes = double(blocks) * threads;
  float ms = time_ms([&] { hipLaunchKernelGGL(k_fma, dim3(blocks), dim3(threads), 0, 0, out, 0.999f, 0.001f); });
  printf("v_fma_f32        %8.3f ms  %7.2f T lane-ops/s\n", ms, lanes * kIt * 8 / ms / 1e9);
  ms = time_ms([&] { hipLaunchKernelGGL(k_trans<false>, dim3(blocks), dim3(threads), 0, 0, out); });
  printf("v_exp_f32        %8.3f ms  %7.2f T lane-ops/s\n", ms, lanes * kIt * 8 / ms / 1e9);
  ms = time_ms([&] { hipLaunchKernelGGL(k_trans<true>, dim3(blocks), dim3(threads), 0, 0, out); });
  printf("v_rsq_f32        %8.3f ms  %7.2f T lane-ops/s\n", ms, lanes * kIt * 8 / ms / 1e9);
  ms = time_ms([&] { hipLaunchKernelGGL(k_mix<0>, dim3(blocks), dim3(threads), 0, 0, out, 0.999f, 0.001f); });
  printf("4 exp + 0 fma    %8.3f ms\n", ms);
  ms = time_ms([&] { hipLaunchKernelGGL(k_mix<1>, dim3(blocks), dim3(threads), 0, 0, out, 0.999f, 0.001f); });
  printf("4 exp + 8 fma    %8.3f ms\n", ms);
  ms = time_ms([&] { hipLaunchKernelGGL(k_mix<2>, dim3(blocks), dim3(threads), 0, 0, out, 0.999f, 0.001f); });
  printf("4 exp + 16 fma   %8.3f ms\n", ms);
  ms = time_ms([&] { hipLaunchKernelGGL(k_mix<4>, dim3(blocks), dim3(threads), 0, 0, out, 0.999f, 0.001f); });
  printf("4 exp + 32 fma   %8.3f ms\n", ms);
  CHECK(hipFree(out));

  const int lblocks = 4096, lthreads = 1024;
  CHECK(hipMalloc(&out, sizeof(float) * (size_t)lblocks * lthreads));
  const double llanes = double(lblocks) * lthreads;
  const char* lds_names[] = {"", "ds_add_f32", "ds_add_u32", "ds_add_u64", "ds_add_f64"};
  for (int mode = 1; mode < 5; ++mode) {
    auto run = [&] {
      switch (mode) {
        case 1: hipLaunchKernelGGL(k_lds<1>, dim3(lblocks), dim3(lthreads), 0, 0, out); break;
        case 2: hipLaunchKernelGGL(k_lds<2>, dim3(lblocks), dim3(lthreads), 0, 0, out); break;
        case 3: hipLaunchKernelGGL(k_lds<3>, dim3(lblocks), dim3(lthreads), 0, 0, out); break;
        default: hipLaunchKernelGGL(k_lds<4>, dim3(lblocks), dim3(lthreads), 0, 0, out); break;
      }
    };
    ms = time_ms(run);
    printf("%-16s %8.3f ms  %7.2f T lane-ops/s\n", lds_names[mode], ms, llanes * kLdsIt / ms / 1e9);
  }
  CHECK(hipFree(out));

  for (unsigned n : {160000u, 16u << 20}) {
    float* buf = nullptr;
    CHECK(hipMalloc(&buf, sizeof(float) * n));
    CHECK(hipMemset(buf, 0, sizeof(float) * n));
    const int iters = 64;
    ms = time_ms([&] { hipLaunchKernelGGL(k_gatomic, dim3(blocks), dim3(threads), 0, 0, buf, n, iters); });
    std::vector<float> h(n);
    CHECK(hipMemcpy(h.data(), buf, sizeof(float) * n, hipMemcpyDeviceToHost));
    double tot = 0.0;
    for (float v : h) tot += v;
    printf("global atomic f32, %u words: %8.3f ms  %7.2f G atomics/s (sum %.0f)\n", n, ms, lanes * iters / ms / 1e6,
           tot);
    CHECK(hipFree(buf));
  }
  return 0;
}
