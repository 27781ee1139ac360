// Streaming bandwidth probes: the practical HBM ceilings the Chebyshev term kernel is measured
// against, from plain kernels with the same access width (16-byte vectors) and the same
// read/write mix, timed with HIP events on the caller's stream.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "rp.h"

namespace rp {
int mlp_fail(int code, const char *msg);
}

namespace {

using f4 = float __attribute__((ext_vector_type(4)));
constexpr int kUnroll = 4;   // 16-byte vectors per thread, strided by the workgroup size

// kind 0: c = a (one read, one write); 1: c = a + b (two reads, one write); 2: read a only
// (one 16-byte store per workgroup); 3: write c only.
template <int KIND>
__global__ __launch_bounds__(256) void k_stream(const f4 *__restrict__ a, const f4 *__restrict__ b,
                                                f4 *__restrict__ c, int64_t n) {
  const int64_t base = (int64_t)blockIdx.x * 256 * kUnroll + threadIdx.x;
  f4 v[kUnroll];
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) {
    const int64_t i = base + (int64_t)u * 256;
    if (i < n) {
      if (KIND == 0 || KIND == 2) v[u] = a[i];
      else if (KIND == 1) v[u] = a[i] + b[i];
      else v[u] = f4{1.f, 2.f, 3.f, 4.f};
    }
  }
  if (KIND == 2) {
    f4 s = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
      if (base + (int64_t)u * 256 < n) s += v[u];
    // one store per workgroup keeps the loads alive without adding traffic
    if (s.x == 1.2345e-38f) c[blockIdx.x] = s;
    return;
  }
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) {
    const int64_t i = base + (int64_t)u * 256;
    if (i < n) c[i] = v[u];
  }
}

template <int KIND>
void launch(const f4 *a, const f4 *b, f4 *c, int64_t n, hipStream_t st) {
  const int64_t blocks = (n + 256 * kUnroll - 1) / (256 * kUnroll);
  hipLaunchKernelGGL(k_stream<KIND>, dim3((unsigned)blocks), dim3(256), 0, st, a, b, c, n);
}

}  // namespace

extern "C" int rp_probe_stream(int32_t kind, const void *a, const void *b, void *c, int64_t bytes, int32_t reps,
                               double *ms_per_launch, void *hip_stream) {
  if (kind < 0 || kind > 3 || bytes < 16 || bytes % 16 || reps < 1 || !ms_per_launch)
    return rp::mlp_fail(RP_EINVAL, "rp_probe_stream: kind 0..3, bytes a positive multiple of 16, reps >= 1");
  if (bytes / 16 / (256 * kUnroll) >= ((int64_t)1 << 31)) return rp::mlp_fail(RP_EINVAL, "rp_probe_stream: too large");
  if ((kind != 3 && !a) || (kind == 1 && !b) || !c) return rp::mlp_fail(RP_EINVAL, "rp_probe_stream: null pointer");
  hipStream_t st = (hipStream_t)hip_stream;
  const int64_t n = bytes / 16;
  const f4 *A = (const f4 *)a, *B = (const f4 *)b;
  f4 *C = (f4 *)c;
  auto one = [&]() {
    switch (kind) {
      case 0: launch<0>(A, B, C, n, st); break;
      case 1: launch<1>(A, B, C, n, st); break;
      case 2: launch<2>(A, B, C, n, st); break;
      default: launch<3>(A, B, C, n, st); break;
    }
  };
  one();   // warm-up
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return rp::mlp_fail(RP_EDEVICE, "rp_probe_stream: event creation failed");
  }
  (void)hipEventRecord(e0, st);
  for (int r = 0; r < reps; ++r) one();
  (void)hipEventRecord(e1, st);
  float ms = 0.f;
  const hipError_t es = hipEventSynchronize(e1);
  const hipError_t ee = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (es != hipSuccess || ee != hipSuccess || hipGetLastError() != hipSuccess)
    return rp::mlp_fail(RP_EDEVICE, "rp_probe_stream: launch or timing failed");
  *ms_per_launch = ms / reps;
  return RP_OK;
}
