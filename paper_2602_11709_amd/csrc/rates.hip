// Instruction-rate and bandwidth microbenchmark of the GPU (gfx950), the
// denominators of the library's roofline figures.
//
//   xrd_rates [--iters N]
//
// prints one JSON object with, for each instruction class the kernels use,
// the measured rate in lane-operations per second and per compute unit and
// clock (at the nominal 2.4 GHz; the sustained clock may differ):
//   fp32_fma   v_fma_f32 (unpacked: the library is built without packed FP32)
//   fp64_fma   v_fma_f64
//   sin        v_sin_f32 (takes revolutions)
//   exp2       v_exp_f32
//   fract64_add  an FP64 add and v_fract_f64 (FP64-rate operations)
//   sf_term    the mixed structure-factor term as the forward kernel evaluates it
//              (3 FP64 operations for the phase, fract + convert, sin, cos, the
//              weight's exp2 with its FP32 FMA, two FP32 FMA for F and, for
//              dF/ds^2, one product and two FMA), in terms per second
// and the bandwidth of a plain device copy (bytes read + written per second).
// Each kernel keeps 8 independent chains per lane and launches 16 blocks of
// 256 lanes per compute unit, so latency is hidden and only issue rate
// remains; the best of 5 launches counts.  The instruction-class rates price
// a term when the classes issue one after another (their costs add); the
// sf_term figure shows whether they overlap.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>

namespace {

constexpr int kThreads = 256;
constexpr int kChains = 8;

#define HIP_OK(x)                                                                       \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess) {                                                             \
      std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));                      \
      std::exit(1);                                                                     \
    }                                                                                   \
  } while (0)

enum Op { FMA32, FMA64, SIN, EXP2, FRACT64 };

template <int OP>
__global__ __launch_bounds__(kThreads) void k_rate(float *out, int iters, float seed) {
  const int tid = blockIdx.x * kThreads + threadIdx.x;
  float a[kChains];
  double d[kChains];
#pragma unroll
  for (int j = 0; j < kChains; ++j) {
    a[j] = seed * (float)(tid % 97 + j + 1) * 1e-3f;
    d[j] = (double)a[j] + 0.25;
  }
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < kChains; ++j) {
      if constexpr (OP == FMA32) {
        a[j] = __builtin_fmaf(a[j], 0.99999994f, 1e-7f);
      } else if constexpr (OP == FMA64) {
        d[j] = __builtin_fma(d[j], 0.9999999999999999, 1e-16);
      } else if constexpr (OP == SIN) {
        a[j] = __builtin_amdgcn_sinf(a[j]);
      } else if constexpr (OP == EXP2) {
        a[j] = __builtin_amdgcn_exp2f(-a[j]);
      } else {
        // an FP64 add and v_fract_f64: two FP64-rate operations per step
        d[j] = __builtin_amdgcn_fract(d[j] + 0.6180339887498949);
      }
    }
  }
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < kChains; ++j) s += a[j] + (float)d[j];
  out[tid] = s;
}

// The mixed structure-factor term as the forward kernel evaluates it (with
// dF/ds^2): per lane fixed reflections (h, k, l, s^2), per step one atom
// record (x, y, z, B log2 e, log2 occ) uniform over the wavefront, loaded
// through the scalar cache like the kernel's, and per term 3 FP64 operations
// for the phase, v_fract_f64 and the conversion, sin, cos and the weight's
// exp2 (after one FP32 FMA), two FP32 FMA for F and a product and two FMA for
// dF/ds^2.
struct Atom {
  double x, y, z;
  float bl2e, log2occ;
};

__global__ __launch_bounds__(kThreads) void k_term(const Atom *__restrict__ atoms, int n_atoms, float *out) {
  const int tid = blockIdx.x * kThreads + threadIdx.x;
  double h[kChains], k[kChains], l[kChains];
  float s2[kChains], pa[kChains], pb[kChains], qa[kChains], qb[kChains];
#pragma unroll
  for (int j = 0; j < kChains; ++j) {
    h[j] = (double)((tid + j) % 29 - 14);
    k[j] = (double)((tid * 7 + j) % 31 - 15);
    l[j] = (double)((tid * 3 + 5 * j) % 27 - 13);
    s2[j] = 0.01f * (float)((tid + j) % 50);
    pa[j] = pb[j] = qa[j] = qb[j] = 0.f;
  }
  for (int i = 0; i < n_atoms; ++i) {
    const Atom a = atoms[i];
#pragma unroll
    for (int j = 0; j < kChains; ++j) {
      const double t = __builtin_fma(h[j], a.x, __builtin_fma(k[j], a.y, l[j] * a.z));
      const float rho = (float)__builtin_amdgcn_fract(t);
      const float sn = __builtin_amdgcn_sinf(rho);
      const float cs = __builtin_amdgcn_cosf(rho);
      const float w = __builtin_amdgcn_exp2f(__builtin_fmaf(-a.bl2e, s2[j], a.log2occ));
      pa[j] = __builtin_fmaf(w, cs, pa[j]);
      pb[j] = __builtin_fmaf(w, sn, pb[j]);
      const float bw = a.bl2e * w;
      qa[j] = __builtin_fmaf(bw, cs, qa[j]);
      qb[j] = __builtin_fmaf(bw, sn, qb[j]);
    }
  }
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < kChains; ++j) s += pa[j] + pb[j] + qa[j] + qb[j];
  out[tid] = s;
}

__global__ __launch_bounds__(kThreads) void k_copy(const float4 *__restrict__ src, float4 *__restrict__ dst,
                                                   size_t n) {
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kThreads)
    dst[i] = src[i];
}

// Best of five timed launches (after one untimed) of ``launch``, in ms.
template <class F>
float best_ms(F &&launch) {
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  launch(0);
  HIP_OK(hipGetLastError());
  float best = 1e30f;
  for (int r = 0; r < 5; ++r) {
    HIP_OK(hipEventRecord(e0, 0));
    launch(r + 1);
    HIP_OK(hipEventRecord(e1, 0));
    HIP_OK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_OK(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best) best = ms;
  }
  HIP_OK(hipEventDestroy(e0));
  HIP_OK(hipEventDestroy(e1));
  return best;
}

// Lane-operations (steps of each chain) per second.
template <int OP>
double time_rate(int n_cu, int iters, float *out) {
  const int blocks = n_cu * 16;
  const float ms = best_ms([&](int r) {
    hipLaunchKernelGGL(k_rate<OP>, dim3(blocks), dim3(kThreads), 0, 0, out, iters, 1.0f + r);
  });
  return (double)blocks * kThreads * iters * kChains / (ms * 1e-3);
}

}  // namespace

int main(int argc, char **argv) {
  int iters = 2048;
  for (int i = 1; i < argc; ++i)
    if (!std::strcmp(argv[i], "--iters") && i + 1 < argc) iters = std::atoi(argv[++i]);
  if (iters < 1 || iters > (1 << 20)) {
    std::fprintf(stderr, "--iters must lie in [1, 2^20]\n");
    return 2;
  }
  hipDeviceProp_t prop;
  HIP_OK(hipGetDeviceProperties(&prop, 0));
  const int n_cu = prop.multiProcessorCount;
  float *out = nullptr;
  HIP_OK(hipMalloc(&out, sizeof(float) * (size_t)n_cu * 16 * kThreads));
  const double clk = 2.4e9;
  const double per = 1.0 / (n_cu * clk);
  const double fma32 = time_rate<FMA32>(n_cu, iters, out);
  const double fma64 = time_rate<FMA64>(n_cu, iters, out);
  const double sn = time_rate<SIN>(n_cu, iters, out);
  const double ex = time_rate<EXP2>(n_cu, iters, out);
  const double fr = 2.0 * time_rate<FRACT64>(n_cu, iters, out);
  // terms: n_atoms atom records, every lane's 8 reflections against each
  const int n_atoms = iters / 4 > 0 ? iters / 4 : 1;
  Atom *atoms = nullptr;
  {
    Atom *host = (Atom *)std::malloc(sizeof(Atom) * (size_t)n_atoms);
    if (!host) return 1;
    for (int i = 0; i < n_atoms; ++i) {
      host[i].x = 0.001 * (i % 997);
      host[i].y = 0.0007 * (i % 1009);
      host[i].z = 0.0013 * (i % 761);
      host[i].bl2e = 0.5f + 0.001f * (float)(i % 100);
      host[i].log2occ = -0.01f * (float)(i % 7);
    }
    HIP_OK(hipMalloc(&atoms, sizeof(Atom) * (size_t)n_atoms));
    HIP_OK(hipMemcpy(atoms, host, sizeof(Atom) * (size_t)n_atoms, hipMemcpyHostToDevice));
    std::free(host);
  }
  const int tblocks = n_cu * 16;
  const float tms = best_ms([&](int) {
    hipLaunchKernelGGL(k_term, dim3(tblocks), dim3(kThreads), 0, 0, atoms, n_atoms, out);
  });
  const double term = (double)tblocks * kThreads * kChains * n_atoms / (tms * 1e-3);
  HIP_OK(hipFree(atoms));
  HIP_OK(hipFree(out));
  // device copy of 1 GiB (float4 per lane)
  const size_t bytes = (size_t)1 << 30, n4 = bytes / sizeof(float4);
  float4 *src = nullptr, *dst = nullptr;
  HIP_OK(hipMalloc(&src, bytes));
  HIP_OK(hipMalloc(&dst, bytes));
  HIP_OK(hipMemset(src, 0, bytes));
  const int cblocks = n_cu * 8;
  const float best = best_ms([&](int) {
    hipLaunchKernelGGL(k_copy, dim3(cblocks), dim3(kThreads), 0, 0, src, dst, n4);
  });
  HIP_OK(hipFree(src));
  HIP_OK(hipFree(dst));
  const double copy_bps = 2.0 * (double)bytes / (best * 1e-3);
  std::printf(
      "{\"device\": \"%s\", \"compute_units\": %d, \"nominal_clock_hz\": %.4g, \"iters\": %d, "
      "\"per_s\": {\"fp32_fma\": %.6g, \"fp64_fma\": %.6g, \"sin\": %.6g, \"exp2\": %.6g, "
      "\"fract64_add\": %.6g, \"sf_term\": %.6g}, "
      "\"per_cu_clk\": {\"fp32_fma\": %.4g, \"fp64_fma\": %.4g, \"sin\": %.4g, \"exp2\": %.4g, "
      "\"fract64_add\": %.4g, \"sf_term\": %.4g}, \"copy_bytes_per_s\": %.6g}\n",
      prop.gcnArchName, n_cu, clk, iters, fma32, fma64, sn, ex, fr, term, fma32 * per, fma64 * per, sn * per,
      ex * per, fr * per, term * per, copy_bps);
  return 0;
}
