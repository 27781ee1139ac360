// Learned control variate for the Monte Carlo trace: a small MLP g(Omega, B) trained on
// single-wavepacket yields phi_S that the propagation itself produced, used as a control
// variate for the sample mean of Eq. 18 (the estimate stays unbiased because the network,
// its coefficient beta and its mean mu are fixed independently of the evaluation samples).
//
// Network: x (features) -> [Linear, GELU] x depth -> Linear -> scalar.  FP32 master
// weights; every hidden-layer product runs on MFMA (v_mfma_f32_16x16x16_bf16, inputs
// rounded to BF16, FP32 accumulation).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>

#include "rp.h"

namespace rp {
int mlp_fail(int code, const char *msg);
}

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (inputs are finite).
__device__ __forceinline__ short to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// C[m][n] = sum_k A(m, k) B(k, n) (+ bias[n]), A(m, k) = A[m*sam + k*sak], B(k, n) = B[k*sbk + n*sbn],
// on the 16x16x16 BF16 MFMA.
// Epilogue: if Z != null store the pre-activation; if H != null store GELU of it; if
// ACC, C is added to the existing contents (gradient accumulation is not used: plain store).
struct GemmArgs {
  const float *A, *B, *bias;
  float *Z, *H;
  int64_t M, N, K;
  int64_t sam, sak, sbk, sbn, ldc;
};

// A workgroup (4 waves) computes a 32 x 32 tile of C: wave w the 16 x 16 quarter (w / 2, w % 2).
// Per step of 32 in K, the workgroup stages the 32 x 32 slices of A and B in LDS once, rounded
// to BF16 (each element is loaded and converted once and used by the two waves that need it),
// then every wave runs two 16x16x16 MFMAs from LDS.  Global loads run along the operand's
// unit-stride dimension (sak or sam for A, sbn or sbk for B), so they are coalesced for the
// plain and the transposed operands of the forward and backward passes.  The sum over K runs in
// the same order as one MFMA per 16 values of K.
constexpr int kGT = 32;            // C tile edge and K step
constexpr int kGP = kGT + 8;       // LDS row length in BF16 values (padding against bank conflicts)

__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  __shared__ short As[kGT][kGP];   // As[m][k]
  __shared__ short Bs[kGT][kGP];   // Bs[n][k]
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t tiles_n = (g.N + kGT - 1) / kGT;
  const int64_t tm = blockIdx.x / tiles_n, tn = blockIdx.x - tm * tiles_n;
  const int64_t m0 = tm * kGT, n0 = tn * kGT;
  const bool a_k_fast = g.sak == 1, b_n_fast = g.sbn == 1;
  const int wm = (w >> 1) * 16, wn = (w & 1) * 16;
  const int kq = 4 * (lane >> 4);
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int64_t k0 = 0; k0 < g.K; k0 += kGT) {
    // 1024 values of each operand slice, four per thread, the unit-stride index fastest
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = q * 256 + t;
      const int fast = e & (kGT - 1), slow = e >> 5;
      {
        const int mm = a_k_fast ? slow : fast, kk = a_k_fast ? fast : slow;
        const int64_t m = m0 + mm, k = k0 + kk;
        As[mm][kk] = to_bf16((m < g.M && k < g.K) ? g.A[m * g.sam + k * g.sak] : 0.f);
      }
      {
        const int nn = b_n_fast ? fast : slow, kk = b_n_fast ? slow : fast;
        const int64_t n = n0 + nn, k = k0 + kk;
        Bs[nn][kk] = to_bf16((n < g.N && k < g.K) ? g.B[k * g.sbk + n * g.sbn] : 0.f);
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kGT; kk += 16) {
      bf16x4 a, b;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        a[i] = As[wm + (lane & 15)][kk + kq + i];
        b[i] = Bs[wn + (lane & 15)][kk + kq + i];
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  // Result layout: lane l, register i -> row 4*(l/16) + i, column l % 16 of the wave's tile.
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t r = m0 + wm + kq + i, c = n0 + wn + (lane & 15);
    if (r < g.M && c < g.N) {
      float z = acc[i] + (g.bias ? g.bias[c] : 0.f);
      if (g.Z) g.Z[r * g.ldc + c] = z;
      if (g.H) g.H[r * g.ldc + c] = gelu(z);
    }
  }
}

// Output layer y[r] = sum_j H[r][j] w[j] + b (one wave per row), optional loss gradient
// dy = 2 (y - t) / rows and per-row squared error.
struct OutArgs {
  const float *H, *w, *b, *t;
  float *y, *dy, *err;
  int64_t rows, width;
};

__global__ __launch_bounds__(256) void k_out(OutArgs o) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= o.rows) return;
  float s = 0.f;
  for (int64_t j = lane; j < o.width; j += 64) s += o.H[r * o.width + j] * o.w[j];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) {
    const float y = s + o.b[0];
    o.y[r] = y;
    if (o.t) {
      const float e = y - o.t[r];
      o.dy[r] = 2.0f * e / (float)o.rows;
      o.err[r] = e * e;
    }
  }
}

// dZ[r][j] = (dy[r] w[j]) * gelu'(Z[r][j])  (gradient through the output layer and the
// last activation), or dZ = dH * gelu'(Z) when dy is null.
struct ActArgs {
  const float *dy, *w, *dH, *Z;
  float *dZ;
  int64_t rows, width;
};

__global__ __launch_bounds__(256) void k_act_back(ActArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.rows * a.width) return;
  const int64_t r = i / a.width, j = i - r * a.width;
  const float up = a.dy ? a.dy[r] * a.w[j] : a.dH[i];
  a.dZ[i] = up * gelu_grad(a.Z[i]);
}

// Column sums over rows: out[j] = sum_r X[r][j] * (v ? v[r] : 1)  (bias gradients and the
// output-weight gradient), one thread per column, FP32.
struct ColArgs {
  const float *X, *v;
  float *out;
  int64_t rows, cols;
};

// Column sums out[j] = sum_r X[r][j] v[r] (v = 1 when null).  A workgroup of 16 waves takes
// 64 columns: the lanes of a wave are the columns (each row segment one coalesced 256-byte
// load), wave w the rows w, w + 16, ...; the 16 wave sums are then added in LDS in a fixed
// order, so the result does not depend on scheduling.
constexpr int kColWaves = 16;
__global__ __launch_bounds__(64 * kColWaves) void k_colsum(ColArgs c) {
  __shared__ float part[kColWaves][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t j = (int64_t)blockIdx.x * 64 + lane;
  float s = 0.f;
  if (j < c.cols)
    for (int64_t r = w; r < c.rows; r += kColWaves) s += c.X[r * c.cols + j] * (c.v ? c.v[r] : 1.0f);
  part[w][lane] = s;
  __syncthreads();
  if (w == 0 && j < c.cols) {
    float t = 0.f;
    for (int k = 0; k < kColWaves; ++k) t += part[k][lane];
    c.out[j] = t;
  }
}

// The sum of one column (cols == 1): threads over rows, then a tree in LDS.
__global__ __launch_bounds__(1024) void k_sum1(ColArgs c) {
  __shared__ float part[1024];
  float s = 0.f;
  for (int64_t r = threadIdx.x; r < c.rows; r += 1024) s += c.X[r] * (c.v ? c.v[r] : 1.0f);
  part[threadIdx.x] = s;
  __syncthreads();
  for (int h = 512; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) c.out[0] = part[0];
}

static void colsum(const ColArgs &c, hipStream_t st) {
  if (c.cols == 1)
    hipLaunchKernelGGL(k_sum1, dim3(1), dim3(1024), 0, st, c);
  else
    hipLaunchKernelGGL(k_colsum, dim3((unsigned)((c.cols + 63) / 64)), dim3(64 * kColWaves), 0, st, c);
}

// Adam (Kingma & Ba) on the packed FP32 parameters.
struct AdamArgs {
  float *p, *m, *v;
  const float *g;
  int64_t n;
  float lr, b1, b2, eps, c1, c2;   // c1 = 1/(1-b1^t), c2 = 1/(1-b2^t)
};

__global__ __launch_bounds__(256) void k_adam(AdamArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const float g = a.g[i];
  const float m = a.b1 * a.m[i] + (1.f - a.b1) * g;
  const float v = a.b2 * a.v[i] + (1.f - a.b2) * g * g;
  a.m[i] = m;
  a.v[i] = v;
  a.p[i] -= a.lr * (m * a.c1) / (sqrtf(v * a.c2) + a.eps);
}

// Features of (sample, field): the unit vectors n(Omega_k) (Eq. 16) of every nucleus and
// log(B/mT + 0.05); rows ordered field-major, zero padded to n_in_pad columns.  With a nonzero
// rot_seed every azimuth of row r is advanced by the same angle 2 pi u_r: a rotation of all
// nuclear directions about the field axis, under which the yield is invariant (H, P_S and the
// singlet commute with the total J_z), used to augment training data.
struct FeatArgs {
  const double *angles, *B;
  float *x;
  int64_t M;
  int32_t N, nB, n_in_pad, layout;
  uint64_t rot_seed;
};

// u in (0, 1) from SplitMix64 (Steele, Lea & Flood 2014) of seed + (r + 1) * golden gamma.
__device__ __forceinline__ double splitmix_unit(uint64_t seed, uint64_t r) {
  uint64_t z = seed + (r + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return ((double)(z >> 11) + 0.5) * 0x1.0p-53;
}

__global__ __launch_bounds__(256) void k_features(FeatArgs f) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t rows = (int64_t)f.nB * f.M;
  if (i >= rows * f.n_in_pad) return;
  const int64_t r = i / f.n_in_pad;
  const int c = (int)(i - r * f.n_in_pad);
  const int64_t b = f.layout == 0 ? r / f.M : r % f.nB;
  const int64_t s = f.layout == 0 ? r - b * f.M : f.layout == 1 ? r / f.nB : r;
  float v = 0.f;
  if (c < 3 * f.N) {
    const int k = c / 3, q = c - 3 * k;
    const double ct = f.angles[(s * f.N + k) * 2];
    double ph = f.angles[(s * f.N + k) * 2 + 1];
    if (f.rot_seed) ph += 6.283185307179586 * splitmix_unit(f.rot_seed, (uint64_t)r);
    const double st = sqrt(fmax(0.0, 1.0 - ct * ct));
    v = (float)(q == 0 ? st * cos(ph) : q == 1 ? st * sin(ph) : ct);
  } else if (c == 3 * f.N) {
    v = (float)log(fabs(f.B[b]) + 0.05);
  }
  f.x[i] = v;
}

// Per-field standardisation of training targets: rows q = s * nB + b (s < n_rows, field b);
// mean and standard deviation (1/n normalisation) of field b over its first n_fit rows; every
// row of the field becomes (phi - mean) / std (std 1 when it is 0).  One workgroup per field.
struct StdArgs {
  const double *phi;
  float *t;
  int64_t nB, n_rows, n_fit;
};

__device__ __forceinline__ double wg_sum(double v, double *lds) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) lds[w] = v;
  __syncthreads();
  const double t = lds[0] + lds[1] + lds[2] + lds[3];
  __syncthreads();
  return t;
}

__global__ __launch_bounds__(256) void k_standardize(StdArgs a) {
  __shared__ double lds[4];
  const int64_t b = blockIdx.x;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < a.n_fit; i += 256) s += a.phi[i * a.nB + b];
  const double mean = wg_sum(s, lds) / (double)a.n_fit;
  double q = 0.0;
  for (int64_t i = threadIdx.x; i < a.n_fit; i += 256) {
    const double d = a.phi[i * a.nB + b] - mean;
    q += d * d;
  }
  double sd = sqrt(wg_sum(q, lds) / (double)a.n_fit);
  if (sd == 0.0) sd = 1.0;
  for (int64_t i = threadIdx.x; i < a.n_rows; i += 256) a.t[i * a.nB + b] = (float)((a.phi[i * a.nB + b] - mean) / sd);
}

// Mean squared error of y against t over rows, accumulated in FP64 by one workgroup.
__global__ __launch_bounds__(256) void k_mse(const float *y, const float *t, int64_t rows, double *out) {
  __shared__ double lds[4];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < rows; i += 256) {
    const double e = (double)y[i] - (double)t[i];
    s += e * e;
  }
  const double tot = wg_sum(s, lds);
  if (threadIdx.x == 0) *out = tot / (double)rows;
}

unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

struct Layout {
  int64_t in_pad, width, depth;
  int64_t off_W[8], off_b[8], off_w, off_bo, total;
};

bool layout_of(int32_t n_in, int32_t width, int32_t depth, Layout &L) {
  if (n_in < 1 || width < 16 || width % 16 || depth < 1 || depth > 8) return false;
  L.in_pad = (n_in + 15) / 16 * 16;
  L.width = width;
  L.depth = depth;
  int64_t o = 0, fan = L.in_pad;
  for (int l = 0; l < depth; ++l) {
    L.off_W[l] = o;
    o += fan * width;
    L.off_b[l] = o;
    o += width;
    fan = width;
  }
  L.off_w = o;
  o += width;
  L.off_bo = o;
  o += 1;
  L.total = o;
  return true;
}

// Workspace per row: depth pre-activations and activations, two gradient buffers, y, dy, err.
int64_t ws_floats(const Layout &L, int64_t rows) {
  return rows * (2 * L.depth * L.width + 2 * L.width + 3) + L.total;
}

void gemm(const float *A, int64_t sam, int64_t sak, const float *B, int64_t sbk, int64_t sbn, const float *bias,
          float *Z, float *H, int64_t M, int64_t N, int64_t K, hipStream_t st) {
  GemmArgs g{A, B, bias, Z, H, M, N, K, sam, sak, sbk, sbn, N};
  const int64_t tiles = ((M + kGT - 1) / kGT) * ((N + kGT - 1) / kGT);
  hipLaunchKernelGGL(k_gemm, dim3((unsigned)tiles), dim3(256), 0, st, g);
}

// Forward pass; returns pointer to y inside the workspace.
float *forward(const Layout &L, const float *P, const float *x, int64_t rows, float *ws, const float *t,
               hipStream_t st) {
  float *Zs = ws, *Hs = ws + rows * L.depth * L.width;
  const float *in = x;
  int64_t fan = L.in_pad;
  for (int l = 0; l < L.depth; ++l) {
    float *Z = Zs + rows * l * L.width, *H = Hs + rows * l * L.width;
    gemm(in, fan, 1, P + L.off_W[l], L.width, 1, P + L.off_b[l], Z, H, rows, L.width, fan, st);
    in = H;
    fan = L.width;
  }
  float *tail = ws + rows * (2 * L.depth * L.width + 2 * L.width);
  float *y = tail, *dy = tail + rows, *err = tail + 2 * rows;
  OutArgs o{in, P + L.off_w, P + L.off_bo, t, y, dy, err, rows, L.width};
  hipLaunchKernelGGL(k_out, dim3(blocks(rows * 64)), dim3(256), 0, st, o);
  return y;
}

}  // namespace

// ============================================================================= C ABI
using rp::mlp_fail;

extern "C" int64_t rp_mlp_param_count(int32_t n_in, int32_t width, int32_t depth) {
  Layout L;
  if (!layout_of(n_in, width, depth, L)) return -1;
  return L.total;
}

extern "C" int64_t rp_mlp_workspace_floats(int32_t n_in, int32_t width, int32_t depth, int64_t rows) {
  Layout L;
  if (!layout_of(n_in, width, depth, L) || rows < 0) return -1;
  return ws_floats(L, rows);
}

extern "C" int rp_mlp_features(const double *angles, int64_t M, int32_t N, const double *B_mT, int32_t nB,
                               int32_t n_in_pad, int32_t layout, uint64_t rot_seed, float *x, void *hip_stream) {
  if (M < 0 || N < 0 || nB < 0 || n_in_pad < 3 * N + 1) return mlp_fail(RP_EINVAL, "bad feature sizes");
  if (layout < 0 || layout > 2) return mlp_fail(RP_EINVAL, "layout must be 0, 1 or 2");
  if (M == 0 || nB == 0) return RP_OK;
  if (!angles || !B_mT || !x) return mlp_fail(RP_EINVAL, "null pointer");
  FeatArgs f{angles, B_mT, x, M, N, nB, n_in_pad, layout, rot_seed};
  hipLaunchKernelGGL(k_features, dim3(blocks((int64_t)nB * M * n_in_pad)), dim3(256), 0,
                     (hipStream_t)hip_stream, f);
  return hipGetLastError() == hipSuccess ? RP_OK : mlp_fail(RP_EDEVICE, "feature kernel launch failed");
}

extern "C" int rp_mlp_forward(int32_t n_in, int32_t width, int32_t depth, const float *params, const float *x,
                              int64_t rows, float *y, float *workspace, void *hip_stream) {
  Layout L;
  if (!layout_of(n_in, width, depth, L)) return mlp_fail(RP_EINVAL, "bad network shape");
  if (rows < 0) return mlp_fail(RP_EINVAL, "rows < 0");
  if (rows == 0) return RP_OK;
  if (!params || !x || !y || !workspace) return mlp_fail(RP_EINVAL, "null pointer");
  hipStream_t st = (hipStream_t)hip_stream;
  float *yo = forward(L, params, x, rows, workspace, nullptr, st);
  if (hipMemcpyAsync(y, yo, rows * sizeof(float), hipMemcpyDeviceToDevice, st) != hipSuccess)
    return mlp_fail(RP_EDEVICE, "copy of outputs failed");
  return hipGetLastError() == hipSuccess ? RP_OK : mlp_fail(RP_EDEVICE, "forward launch failed");
}

extern "C" int rp_mlp_train_step(int32_t n_in, int32_t width, int32_t depth, float *params, float *adam_m,
                                 float *adam_v, int64_t step, const float *x, const float *target, int64_t rows,
                                 float lr, float *grad_out, float *sq_err, float *workspace, void *hip_stream) {
  Layout L;
  if (!layout_of(n_in, width, depth, L)) return mlp_fail(RP_EINVAL, "bad network shape");
  if (rows < 1 || step < 1 || !(lr >= 0.f)) return mlp_fail(RP_EINVAL, "rows, step or lr out of range");
  if (!params || !adam_m || !adam_v || !x || !target || !workspace) return mlp_fail(RP_EINVAL, "null pointer");
  hipStream_t st = (hipStream_t)hip_stream;
  const int64_t W = L.width, R = rows;
  float *Zs = workspace, *Hs = workspace + R * L.depth * W;
  float *dA = workspace + R * 2 * L.depth * W, *dB = dA + R * W;
  float *tail = dB + R * W;
  float *dy = tail + R, *err = tail + 2 * R;
  float *G = tail + 3 * R;   // gradient, packed like the parameters
  forward(L, params, x, R, workspace, target, st);
  // output layer: dw = H_last^T dy, db = sum dy
  const float *Hl = Hs + R * (L.depth - 1) * W;
  ColArgs c1{Hl, dy, G + L.off_w, R, W};
  colsum(c1, st);
  ColArgs c2{dy, nullptr, G + L.off_bo, R, 1};
  colsum(c2, st);
  // last hidden layer: dZ = (dy w^T) * gelu'(Z)
  ActArgs a{dy, params + L.off_w, nullptr, Zs + R * (L.depth - 1) * W, dA, R, W};
  hipLaunchKernelGGL(k_act_back, dim3(blocks(R * W)), dim3(256), 0, st, a);
  for (int l = L.depth - 1; l >= 0; --l) {
    const float *inp = l ? Hs + R * (l - 1) * W : x;
    const int64_t fan = l ? W : L.in_pad;
    // dW_l = in^T dZ  (fan x W), K = rows
    gemm(inp, 1, fan, dA, W, 1, nullptr, G + L.off_W[l], nullptr, fan, W, R, st);
    ColArgs cb{dA, nullptr, G + L.off_b[l], R, W};
    colsum(cb, st);
    if (l) {
      // dH_{l-1} = dZ W_l^T  (rows x W), then dZ_{l-1} = dH * gelu'(Z_{l-1})
      gemm(dA, W, 1, params + L.off_W[l], 1, W, nullptr, dB, nullptr, R, W, W, st);
      ActArgs ab{nullptr, nullptr, dB, Zs + R * (l - 1) * W, dA, R, W};
      hipLaunchKernelGGL(k_act_back, dim3(blocks(R * W)), dim3(256), 0, st, ab);
    }
  }
  if (grad_out && hipMemcpyAsync(grad_out, G, L.total * sizeof(float), hipMemcpyDeviceToDevice, st) != hipSuccess)
    return mlp_fail(RP_EDEVICE, "gradient copy failed");
  if (sq_err && hipMemcpyAsync(sq_err, err, R * sizeof(float), hipMemcpyDeviceToDevice, st) != hipSuccess)
    return mlp_fail(RP_EDEVICE, "error copy failed");
  const float b1 = 0.9f, b2 = 0.999f;
  AdamArgs ad{params, adam_m, adam_v, G, L.total, lr, b1, b2, 1e-8f,
              (float)(1.0 / (1.0 - std::pow(0.9, (double)step))), (float)(1.0 / (1.0 - std::pow(0.999, (double)step)))};
  if (lr > 0.f) hipLaunchKernelGGL(k_adam, dim3(blocks(L.total)), dim3(256), 0, st, ad);
  return hipGetLastError() == hipSuccess ? RP_OK : mlp_fail(RP_EDEVICE, "training launch failed");
}

extern "C" int rp_mlp_standardize(const double *phi, int32_t nB, int64_t n_rows, int64_t n_fit, float *target,
                                  void *hip_stream) {
  if (nB < 1 || n_rows < 1 || n_fit < 1 || n_fit > n_rows) return mlp_fail(RP_EINVAL, "bad standardisation sizes");
  if (!phi || !target) return mlp_fail(RP_EINVAL, "null pointer");
  StdArgs a{phi, target, nB, n_rows, n_fit};
  hipLaunchKernelGGL(k_standardize, dim3((unsigned)nB), dim3(256), 0, (hipStream_t)hip_stream, a);
  return hipGetLastError() == hipSuccess ? RP_OK : mlp_fail(RP_EDEVICE, "standardisation launch failed");
}

extern "C" int rp_mlp_loss(int32_t n_in, int32_t width, int32_t depth, const float *params, const float *x,
                           const float *target, int64_t rows, double *mse, float *workspace, void *hip_stream) {
  Layout L;
  if (!layout_of(n_in, width, depth, L)) return mlp_fail(RP_EINVAL, "bad network shape");
  if (rows < 1) return mlp_fail(RP_EINVAL, "rows < 1");
  if (!params || !x || !target || !mse || !workspace) return mlp_fail(RP_EINVAL, "null pointer");
  hipStream_t st = (hipStream_t)hip_stream;
  float *y = forward(L, params, x, rows, workspace, nullptr, st);
  hipLaunchKernelGGL(k_mse, dim3(1), dim3(256), 0, st, (const float *)y, target, rows, mse);
  return hipGetLastError() == hipSuccess ? RP_OK : mlp_fail(RP_EDEVICE, "loss launch failed");
}
