// Streaming bandwidth probes: the practical HBM ceilings the Chebyshev term kernel is measured
// against, from plain kernels with the same access width (16-byte vectors) and the same
// read/write mix, timed with HIP events on the caller's stream; the fastest of three variants
// (one or four vectors per thread, plain or non-temporal) counts.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "rp.h"

namespace rp {
int mlp_fail(int code, const char *msg);
}

namespace {

using f4 = float __attribute__((ext_vector_type(4)));

// kind 0: c = a (one read, one write); 1: c = a + b (two reads, one write); 2: read a only
// (a store only where the sum has an impossible value, which keeps the loads alive); 3: write
// c only.  U 16-byte vectors per thread, strided by the workgroup size; NT: non-temporal.
template <int KIND, int U, bool NT>
__global__ __launch_bounds__(256) void k_stream(const f4 *__restrict__ a, const f4 *__restrict__ b,
                                                f4 *__restrict__ c, int64_t n) {
  const int64_t base = (int64_t)blockIdx.x * 256 * U + threadIdx.x;
  f4 v[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t i = base + (int64_t)u * 256;
    if (i < n) {
      if (KIND == 3) {
        v[u] = f4{1.f, 2.f, 3.f, 4.f};
      } else {
        v[u] = NT ? __builtin_nontemporal_load(a + i) : a[i];
        if (KIND == 1) v[u] += NT ? __builtin_nontemporal_load(b + i) : b[i];
      }
    }
  }
  if (KIND == 2) {
    f4 s = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (base + (int64_t)u * 256 < n) s += v[u];
    if (s.x == 1.2345e-38f) c[blockIdx.x] = s;
    return;
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t i = base + (int64_t)u * 256;
    if (i < n) {
      if (NT) __builtin_nontemporal_store(v[u], c + i);
      else c[i] = v[u];
    }
  }
}

template <int KIND, int U, bool NT>
void launch(const f4 *a, const f4 *b, f4 *c, int64_t n, hipStream_t st) {
  const int64_t blocks = (n + 256 * U - 1) / (256 * U);
  hipLaunchKernelGGL((k_stream<KIND, U, NT>), dim3((unsigned)blocks), dim3(256), 0, st, a, b, c, n);
}

// The variants tried per kind (the fastest is reported): one vector per thread; four per
// thread; four per thread with non-temporal accesses.
template <int KIND>
void launch_variant(int var, const f4 *a, const f4 *b, f4 *c, int64_t n, hipStream_t st) {
  if (var == 0) launch<KIND, 1, false>(a, b, c, n, st);
  else if (var == 1) launch<KIND, 4, false>(a, b, c, n, st);
  else launch<KIND, 4, true>(a, b, c, n, st);
}

}  // namespace

extern "C" int rp_probe_stream(int32_t kind, const void *a, const void *b, void *c, int64_t bytes, int32_t reps,
                               double *ms_per_launch, void *hip_stream) {
  if (kind < 0 || kind > 3 || bytes < 16 || bytes % 16 || reps < 1 || !ms_per_launch)
    return rp::mlp_fail(RP_EINVAL, "rp_probe_stream: kind 0..3, bytes a positive multiple of 16, reps >= 1");
  if (bytes / 16 / 256 >= ((int64_t)1 << 31)) return rp::mlp_fail(RP_EINVAL, "rp_probe_stream: too large");
  if ((kind != 3 && !a) || (kind == 1 && !b) || !c) return rp::mlp_fail(RP_EINVAL, "rp_probe_stream: null pointer");
  hipStream_t st = (hipStream_t)hip_stream;
  const int64_t n = bytes / 16;
  const f4 *A = (const f4 *)a, *B = (const f4 *)b;
  f4 *C = (f4 *)c;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return rp::mlp_fail(RP_EDEVICE, "rp_probe_stream: event creation failed");
  }
  double best = -1.0;
  for (int var = 0; var < 3; ++var) {
    auto one = [&]() {
      switch (kind) {
        case 0: launch_variant<0>(var, A, B, C, n, st); break;
        case 1: launch_variant<1>(var, A, B, C, n, st); break;
        case 2: launch_variant<2>(var, A, B, C, n, st); break;
        default: launch_variant<3>(var, A, B, C, n, st); break;
      }
    };
    one();   // warm-up
    (void)hipEventRecord(e0, st);
    for (int r = 0; r < reps; ++r) one();
    (void)hipEventRecord(e1, st);
    float ms = 0.f;
    const hipError_t es = hipEventSynchronize(e1);
    const hipError_t ee = hipEventElapsedTime(&ms, e0, e1);
    if (es != hipSuccess || ee != hipSuccess || hipGetLastError() != hipSuccess) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return rp::mlp_fail(RP_EDEVICE, "rp_probe_stream: launch or timing failed");
    }
    if (best < 0.0 || ms / reps < best) best = ms / reps;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms_per_launch = best;
  return RP_OK;
}
