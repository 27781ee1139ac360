// librp: HIP kernels for gfx950 and the C-ABI entry points declared in include/rp.h.
//
// Hot loop: one launch per Chebyshev term applies the matrix-free generator
//   Gh x = ((H + i beta P_S - c) x) / r
// of Eq. 1-4 to every active wavepacket of a chunk, with
//   H x  (e, M) = diag(e, M) x(e, M) + J x(e^3, M)[e = ab, ba]
//                + sum_k f_k x(e ^ flip_i(k), M +- stride_k)       (flip-flop terms a_k/2 (I+ S- + I- S+)),
// writes phi_{n+1} = 2 Gh phi_n - phi_{n-1} over phi_{n-1}, the singlet amplitude
// <S|phi_{n+1}(M)> (times sqrt 2) into a per-term slab, and adds a_{n+1} phi_{n+1}
// to the accumulator of the step.  At the end of each step one launch contracts
// the per-term slabs with the in-step quadrature factor (the exact time integral
// of P_S over the step), and one launch adds the weighted result to phi_S.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <tuple>
#include <mutex>
#include <numeric>
#include <string>
#include <type_traits>
#include <thread>
#include <type_traits>
#include <vector>

#include "kernels.hpp"
#include "plan.hpp"
#include "rp.h"

namespace rp {

// ----------------------------------------------------------------------------- complex helpers
template <typename R>
__device__ __forceinline__ cx<R> cadd(cx<R> a, cx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ cx<R> csub(cx<R> a, cx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ cx<R> cscale(R s, cx<R> a) { return {s * a.x, s * a.y}; }
template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
template <typename R>
__device__ __forceinline__ cx<R> csel(bool c, cx<R> a, cx<R> b) { return {c ? a.x : b.x, c ? a.y : b.y}; }

// Workgroup b of a 1-D grid runs on XCD b % 8.  Give each XCD a contiguous range
// of logical blocks so that all blocks of one wavepacket share that XCD's L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t total) {
  const int64_t q = total >> 3, rem = total & 7;
  const int64_t x = b & 7, slot = b >> 3;
  return x * q + (x < rem ? x : rem) + slot;
}

__device__ __forceinline__ double warp_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the 256 threads of a workgroup (every thread must call it).
__device__ __forceinline__ double block_sum(double v, double *lds) {
  v = warp_sum(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) lds[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) t = lds[0] + lds[1] + lds[2] + lds[3];
  __syncthreads();
  return t;
}

// The tile a workgroup of a tiled launch works on.  In a launch over the jobs of one system
// every job has nbx tiles and job = L / nbx; in the job queue (several systems, unequal Z)
// tile_job maps the tile to its job, whose descriptor holds the job's offsets.  The tile index
// L is also the index of the workgroup's partial sums.
struct TileRef {
  int64_t job, bx, Z, vec, amp;
  int32_t sys, fi;
};
template <bool Q, typename A>
__device__ __forceinline__ TileRef tile_ref(const A &ta, int64_t L, int64_t Z1) {
  TileRef t;
  if constexpr (Q) {
    t.job = __builtin_amdgcn_readfirstlane(ta.tile_job[L]);
    const QJob &j = ta.jobs[t.job];
    t.sys = j.sys;
    t.fi = j.field;
    t.Z = j.Z;
    t.vec = j.vec;
    t.amp = j.amp;
    t.bx = L - j.blk;
  } else {
    t.job = L / ta.nbx;
    t.bx = L - t.job * ta.nbx;
    t.Z = Z1;
    t.vec = t.job * Z1 * 4;
    t.amp = t.job * Z1;
    t.sys = 0;
    t.fi = ta.job_field[t.job];
  }
  return t;
}

// ----------------------------------------------------------------------------- sampler (Eq. 18)
struct SampleArgs {
  double *angles;
  uint64_t seed, first;
  int64_t M;
  int32_t N, mode;
  uint32_t stream;
  int32_t d[RP_MAX_NUCLEI];
  int64_t radix[RP_MAX_NUCLEI];
  uint64_t rows;   // modes 3 and 4: rows of the sign-flip design (samples per group)
};

__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
    const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
    const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

__global__ __launch_bounds__(256) void k_sample(SampleArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.M * a.N) return;
  const int64_t s = i / a.N;
  const int k = (int)(i - s * a.N);
  // Sign-flip designs draw one set of directions per group of `rows` consecutive samples.
  const uint64_t q = a.first + (uint64_t)s;
  const bool design = a.mode >= 3;
  uint64_t c[4] = {design ? q / a.rows : q, (uint64_t)k, 0ull, 0ull};
  philox4x64_10(c, a.seed, (uint64_t)a.stream);
  const double u1 = ((double)(c[0] >> 12) + 0.5) * 0x1p-52;
  const double u2 = ((double)(c[1] >> 12) + 0.5) * 0x1p-52;
  double v0, v1 = 0.0;
  if (a.mode == 0 || design) {
    v0 = 2.0 * u1 - 1.0;
    v1 = 6.283185307179586 * u2;
    if (design) {
      // Row r of the design: antithetic pair (mode 3); the fold-over of the Sylvester-Hadamard
      // matrix of order n = rows / 2, entry (-1)^popcount(r & k), negated for r >= n (mode 4);
      // column k + 1 of the Sylvester-Hadamard matrix of order rows (mode 5).  A -1 maps n_k
      // to -n_k: cos theta -> -cos theta, phi -> phi + pi (mod 2 pi).
      const uint64_t r = q % a.rows;
      bool neg;
      if (a.mode == 3) {
        neg = r == 1;
      } else if (a.mode == 4) {
        const uint64_t n = a.rows >> 1;
        const uint64_t rr = r < n ? r : r - n;
        neg = ((__popcll(rr & (uint64_t)k) & 1) != 0) != (r >= n);
      } else {
        neg = (__popcll(r & (uint64_t)(k + 1)) & 1) != 0;
      }
      if (neg) {
        v0 = -v0;
        v1 = v1 + 3.141592653589793;
        if (v1 >= 6.283185307179586) v1 -= 6.283185307179586;
      }
    }
  } else if (a.mode == 1) {
    int dg = (int)(u1 * (double)a.d[k]);
    v0 = (double)(dg < a.d[k] ? dg : a.d[k] - 1);
  } else {
    v0 = (double)(((a.first + (uint64_t)s) / (uint64_t)a.radix[k]) % (uint64_t)a.d[k]);
  }
  a.angles[2 * i] = v0;
  a.angles[2 * i + 1] = v1;
}

// ----------------------------------------------------------------------------- initial wavepacket
struct CohArgs {
  const double *angles;   // [M][N][2], caller's nucleus order
  cx<double> *tab;        // [M][N][RP_MAX_TWO_I+1], internal nucleus order
  int64_t M;
  int32_t N, mode;
  int32_t two_I[RP_MAX_NUCLEI];   // internal order
  int32_t perm[RP_MAX_NUCLEI];    // caller's index of internal nucleus k
};

// Components <I, I-n | Omega> of the coherent state of Eq. 15:
//   sqrt(C(2I, n)) (cos theta/2)^(2I-n) (sin theta/2)^n exp(i n phi),
// which is the power series of exp(tan(theta/2) e^{i phi} J_-) |I,I> times (cos theta/2)^{2I}.
__global__ __launch_bounds__(256) void k_coherent(CohArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.M * a.N) return;
  const int64_t s = i / a.N;
  const int k = (int)(i - s * a.N);
  const int t = a.two_I[k];
  cx<double> *out = a.tab + i * (RP_MAX_TWO_I + 1);
  const int64_t src = s * a.N + a.perm[k];
  const double v0 = a.angles[2 * src], v1 = a.angles[2 * src + 1];
  if (a.mode == 1) {
    const int dg = (int)v0;
    for (int n = 0; n <= RP_MAX_TWO_I; ++n) out[n] = {n == dg ? 1.0 : 0.0, 0.0};
    return;
  }
  const double ch = sqrt(fmax(0.0, 0.5 * (1.0 + v0)));
  const double sh = sqrt(fmax(0.0, 0.5 * (1.0 - v0)));
  // sqrt of binomial coefficients C(t, n) for t <= 4
  const double sb[5][5] = {{1, 0, 0, 0, 0},
                           {1, 1, 0, 0, 0},
                           {1, 1.4142135623730951, 1, 0, 0},
                           {1, 1.7320508075688772, 1.7320508075688772, 1, 0},
                           {1, 2, 2.449489742783178, 2, 1}};
  for (int n = 0; n <= RP_MAX_TWO_I; ++n) {
    if (n > t) {
      out[n] = {0.0, 0.0};
      continue;
    }
    double mag = sb[t][n];
    for (int q = 0; q < t - n; ++q) mag *= ch;
    for (int q = 0; q < n; ++q) mag *= sh;
    double sn, cs;
    sincos((double)n * v1, &sn, &cs);
    out[n] = {mag * cs, mag * sn};
  }
}

template <typename R>
struct InitArgs {
  cx<R> *psi;                   // [jobs][4Z]
  const cx<double> *tab;        // [M][N][5]
  const int32_t *job_sample;    // [jobs]
  const int32_t *init_map;      // job queue: [tiles][2] = (slot, tile within the slot)
  const QJob *jobs;             // job queue: slot descriptors (offsets, coherent-table row)
  const SysArgs<R> *systab;     // job queue: systems
  int64_t Z;
  int64_t nbx;
  int64_t tiles;
  int32_t njobs, N;
  int32_t stride[RP_MAX_NUCLEI];
  int32_t d[RP_MAX_NUCLEI];
  int64_t vstride;              // elements between jobs; 0 selects 4Z
};

// psi_0 = |S> (x) prod_k |Omega_k>, |S> = (|ab> - |ba>)/sqrt 2 (Eq. 10, 18-19).
template <typename R, bool Q>
__global__ __launch_bounds__(256) void k_init(InitArgs<R> a) {
  const int64_t L = xcd_remap(blockIdx.x, a.tiles);
  int64_t M, Z, off;
  const cx<double> *t;
  int N;
  const int32_t *stride, *d;
  if constexpr (Q) {
    const int64_t job = a.init_map[2 * L];
    const QJob &j = a.jobs[job];
    const SysArgs<R> &sa = a.systab[j.sys];
    M = (int64_t)a.init_map[2 * L + 1] * kBlock + threadIdx.x;
    Z = j.Z;
    off = j.vec;
    t = a.tab + j.tab * (RP_MAX_TWO_I + 1);
    N = sa.N;
    stride = sa.stride;
    d = sa.d;
  } else {
    const int64_t job = L / a.nbx, bx = L - job * a.nbx;
    M = bx * kBlock + threadIdx.x;
    Z = a.Z;
    off = job * (a.vstride ? a.vstride : a.Z * 4);
    t = a.tab + (int64_t)a.job_sample[job] * a.N * (RP_MAX_TWO_I + 1);
    N = a.N;
    stride = a.stride;
    d = a.d;
  }
  if (M >= Z) return;
  cx<double> p = {M_SQRT1_2, 0.0};
  for (int k = 0; k < N; ++k) {
    const int n = (int)((M / stride[k]) % d[k]);
    const cx<double> c = t[k * (RP_MAX_TWO_I + 1) + n];
    p = {p.x * c.x - p.y * c.y, p.x * c.y + p.y * c.x};
  }
  cx<R> *o = a.psi + off + M;   // planes (aa, ab, ba, bb), each Z long
  o[0] = {R(0), R(0)};
  o[Z] = {R(p.x), R(p.y)};
  o[2 * Z] = {R(-p.x), R(-p.y)};
  o[3 * Z] = {R(0), R(0)};
}

// ----------------------------------------------------------------------------- Chebyshev term
template <typename R>
__device__ __forceinline__ void load2(const cx<R> *p, cx<R> &a, cx<R> &b) {
  a = p[0];
  b = p[1];
}
template <>
__device__ __forceinline__ void load2<float>(const cx<float> *p, cx<float> &a, cx<float> &b) {
  const float4 v = *reinterpret_cast<const float4 *>(p);
  a = {v.x, v.y};
  b = {v.z, v.w};
}

// Which step accumulator work a term launch does (see TiledRun::run).
enum TermMode { kFirst = 0, kPlain = 1, kAcc3 = 2 };

// Adds the flip-flop contribution of one spin-1/2 nucleus on radical 1 (r1) or 2, given
// the two partner components it couples to (bit: this nucleus's digit at M).
template <typename R>
__device__ __forceinline__ void flip_half(bool r1, int bit, R f, cx<R> p0, cx<R> p1, cx<R> &y0, cx<R> &y1,
                                          cx<R> &y2, cx<R> &y3) {
  const cx<R> u0 = cscale(f, p0), u1 = cscale(f, p1), z = {R(0), R(0)};
  if (r1) {   // bit 0: (aa, ab) of the partner feed (ba, bb); bit 1: (ba, bb) feed (aa, ab)
    y0 = cadd(y0, csel(bit, u0, z));
    y1 = cadd(y1, csel(bit, u1, z));
    y2 = cadd(y2, csel(bit, z, u0));
    y3 = cadd(y3, csel(bit, z, u1));
  } else {    // bit 0: (aa, ba) feed (ab, bb); bit 1: (ab, bb) feed (aa, ba)
    y0 = cadd(y0, csel(bit, u0, z));
    y2 = cadd(y2, csel(bit, u1, z));
    y1 = cadd(y1, csel(bit, z, u0));
    y3 = cadd(y3, csel(bit, z, u1));
  }
}

// Everything after H x for one nuclear index: diagonal, exchange, i beta P_S, shift and
// scale, recurrence.  Returns the four components of phi_{n+1}.
template <typename R, int MODE>
__device__ __forceinline__ void term_z(const SysArgs<R> &sa, const FieldDev<R> &fp, R h1, R h2, cx<R> x0, cx<R> x1,
                                       cx<R> x2, cx<R> x3, cx<R> o0, cx<R> o1, cx<R> o2, cx<R> o3, cx<R> y0,
                                       cx<R> y1, cx<R> y2, cx<R> y3, cx<R> &z0, cx<R> &z1, cx<R> &z2, cx<R> &z3) {
  // Diagonal: omega (s1 + s2) + s1 h1 + s2 h2 + 2 J s1 s2 with s = +-1/2.
  const R hs = R(0.5) * (h1 + h2), hd = R(0.5) * (h1 - h2), hj = R(0.5) * sa.J;
  y0 = cadd(y0, cscale(fp.omega + hs + hj, x0));
  y1 = cadd(y1, cadd(cscale(hd - hj, x1), cscale(sa.J, x2)));
  y2 = cadd(y2, cadd(cscale(-hd - hj, x2), cscale(sa.J, x1)));
  y3 = cadd(y3, cscale(-fp.omega - hs + hj, x3));
  // i beta P_S x: P_S acts on (ab, ba) as [[1,-1],[-1,1]]/2.
  const cx<R> t = {R(0.5) * (x1.x - x2.x), R(0.5) * (x1.y - x2.y)};
  const cx<R> ibt = {-sa.beta * t.y, sa.beta * t.x};
  y1 = cadd(y1, ibt);
  y2 = csub(y2, ibt);
  const cx<R> c = {fp.c_re, fp.c_im};
  const R s = MODE == kFirst ? fp.s1 : fp.s2;
  z0 = cscale(s, csub(y0, cmul(c, x0)));
  z1 = cscale(s, csub(y1, cmul(c, x1)));
  z2 = cscale(s, csub(y2, cmul(c, x2)));
  z3 = cscale(s, csub(y3, cmul(c, x3)));
  if (MODE != kFirst) {
    z0 = csub(z0, o0);
    z1 = csub(z1, o1);
    z2 = csub(z2, o2);
    z3 = csub(z3, o3);
  }
}

// New accumulator value of one component: first term a_0 phi_0 + a_1 phi_1; every third
// term acc + a_{n-1} phi_{n-1} + a_n phi_n + a_{n+1} phi_{n+1}.
template <typename R, int MODE>
__device__ __forceinline__ cx<R> acc_value(cx<R> am, cx<R> a0, cx<R> ap, cx<R> v, cx<R> o, cx<R> x, cx<R> z) {
  if (MODE == kFirst) return cadd(cmul(am, x), cmul(a0, z));
  return cadd(v, cadd(cadd(cmul(am, o), cmul(a0, x)), cmul(ap, z)));
}

// term_z, then the stores of phi_{n+1}, its singlet amplitude and the accumulator.
template <typename R, int MODE, bool NT>
__device__ __forceinline__ void finish_term(const TermArgs<R> &ta, const SysArgs<R> &sa, const FieldDev<R> &fp,
                                            const TileRef &t, int64_t M, R h1, R h2, cx<R> x0, cx<R> x1,
                                            cx<R> x2, cx<R> x3, cx<R> o0, cx<R> o1, cx<R> o2, cx<R> o3,
                                            cx<R> y0, cx<R> y1, cx<R> y2, cx<R> y3) {
  cx<R> z0, z1, z2, z3;
  term_z<R, MODE>(sa, fp, h1, h2, x0, x1, x2, x3, o0, o1, o2, o3, y0, y1, y2, y3, z0, z1, z2, z3);
  const int64_t Z = t.Z;
  const int64_t e = t.vec + M;
  const int fi = t.fi;
  cx<R> *O = ta.phio + e;
  st_nt<NT>(O, z0);
  st_nt<NT>(O + Z, z1);
  st_nt<NT>(O + 2 * Z, z2);
  st_nt<NT>(O + 3 * Z, z3);
  st_nt<true>(ta.dnext + t.amp + M, csub(z1, z2));
  const cx<R> *cf = ta.coef + (int64_t)fi * ta.n_terms;
  cx<R> *A = ta.acc + e;
  const cx<R> zero = {R(0), R(0)};
  if (MODE == kFirst) {
    const cx<R> a0 = cf[0], a1 = cf[1];
    st_nt<NT>(A, acc_value<R, MODE>(a0, a1, zero, zero, zero, x0, z0));
    st_nt<NT>(A + Z, acc_value<R, MODE>(a0, a1, zero, zero, zero, x1, z1));
    st_nt<NT>(A + 2 * Z, acc_value<R, MODE>(a0, a1, zero, zero, zero, x2, z2));
    st_nt<NT>(A + 3 * Z, acc_value<R, MODE>(a0, a1, zero, zero, zero, x3, z3));
    st_nt<true>(ta.dfirst + t.amp + M, csub(x1, x2));
  } else if (MODE == kAcc3) {
    const cx<R> am = cf[ta.n - 1], a0 = cf[ta.n], ap = cf[ta.n + 1];
    const cx<R> v0 = ld_nt<NT>(A), v1 = ld_nt<NT>(A + Z), v2 = ld_nt<NT>(A + 2 * Z),
                v3 = ld_nt<NT>(A + 3 * Z);
    st_nt<NT>(A, acc_value<R, MODE>(am, a0, ap, v0, o0, x0, z0));
    st_nt<NT>(A + Z, acc_value<R, MODE>(am, a0, ap, v1, o1, x1, z1));
    st_nt<NT>(A + 2 * Z, acc_value<R, MODE>(am, a0, ap, v2, o2, x2, z2));
    st_nt<NT>(A + 3 * Z, acc_value<R, MODE>(am, a0, ap, v3, o3, x3, z3));
  }
}

// One Chebyshev term for systems whose nuclei are ordered spin-1/2 first (strides 2^k) and
// whose higher spins, if any, have strides that are multiples of 256.  The workgroup's 256
// nuclear indices form a tile that holds every partner along the fast axes (stride < 256);
// the tile is staged in LDS and those partners are read from it.  Partners along the slow
// spin-1/2 axes are read from global memory in batches of 8 loads; higher spins follow with
// workgroup-uniform digits.
constexpr int kSlowBatch = 8;   // slow-axis partner loads issued together
template <typename R, int MODE, bool NT, bool Q>
__global__ __launch_bounds__(256) void k_cheb_tile(TermArgs<R> ta, SysArgs<R> sa1) {
  __shared__ cx<R> tile[kBlock * 4];
  __shared__ double lds[4];
  const int64_t L = ta.remap ? xcd_remap(blockIdx.x, ta.tiles) : (int64_t)blockIdx.x;
  const TileRef t = tile_ref<Q>(ta, L, sa1.Z);
  const SysArgs<R> &sa = Q ? ta.systab[t.sys] : sa1;
  const int64_t bx = t.bx;
  const int tid = threadIdx.x;
  const int64_t M = bx * kBlock + tid;
  const int64_t Z = t.Z;
  const bool live = M < Z;
  const FieldDev<R> fp = ta.fields[t.fi];
  const cx<R> *X = ta.phin + t.vec;
  const cx<R> zero = {R(0), R(0)};
  cx<R> x0 = zero, x1 = zero, x2 = zero, x3 = zero, o0 = zero, o1 = zero, o2 = zero, o3 = zero;
  if (live) {
    x0 = X[M];
    x1 = X[Z + M];
    x2 = X[2 * Z + M];
    x3 = X[3 * Z + M];
    if (MODE != kFirst) {
      const cx<R> *O = ta.phio + t.vec + M;
      o0 = ld_nt<NT>(O);
      o1 = ld_nt<NT>(O + Z);
      o2 = ld_nt<NT>(O + 2 * Z);
      o3 = ld_nt<NT>(O + 3 * Z);
    }
  }
  tile[tid] = x0;                 // planar tile: tile[e * 256 + t]
  tile[kBlock + tid] = x1;
  tile[2 * kBlock + tid] = x2;
  tile[3 * kBlock + tid] = x3;
  __syncthreads();
  double nrm = 0.0;
  if (live) {
    cx<R> y0 = zero, y1 = zero, y2 = zero, y3 = zero;
    R h1 = R(0), h2 = R(0);
    const int nh = sa.nhalf;
    const int kf = nh < 8 ? nh : 8;   // spin-1/2 nuclei whose partners lie in the tile
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (k < kf) {
        const int bit = (tid >> k) & 1;
        const int pt = tid ^ (1 << k);
        const bool r1 = sa.rad[k] == 0;
        const R mk = bit ? R(-0.5) : R(0.5);
        if (r1) h1 += sa.a[k] * mk; else h2 += sa.a[k] * mk;
        cx<R> p0, p1;
        if (r1) {
          p0 = tile[(2 * bit) * kBlock + pt];
          p1 = tile[(2 * bit + 1) * kBlock + pt];
        } else {
          p0 = tile[bit * kBlock + pt];
          p1 = tile[(bit + 2) * kBlock + pt];
        }
        flip_half(r1, bit, sa.f[k][0], p0, p1, y0, y1, y2, y3);
      }
    }
    for (int k0 = kf; k0 < nh; k0 += kSlowBatch) {
      cx<R> pa[kSlowBatch], pb[kSlowBatch];
#pragma unroll
      for (int j = 0; j < kSlowBatch; ++j) {
        const int k = k0 + j;
        if (k < nh) {
          const int bit = (int)((M >> k) & 1);
          const int64_t P = M ^ ((int64_t)1 << k);
          // slow axis: every lane of a wave has the same bit, so both loads are coalesced
          const bool r1k = sa.rad[k] == 0;
          const int c0 = r1k ? 2 * bit : bit, c1 = r1k ? 2 * bit + 1 : bit + 2;
          pa[j] = X[c0 * Z + P];
          pb[j] = X[c1 * Z + P];
        }
      }
#pragma unroll
      for (int j = 0; j < kSlowBatch; ++j) {
        const int k = k0 + j;
        if (k < nh) {
          const int bit = (int)((M >> k) & 1);
          const bool r1 = sa.rad[k] == 0;
          const R mk = bit ? R(-0.5) : R(0.5);
          if (r1) h1 += sa.a[k] * mk; else h2 += sa.a[k] * mk;
          flip_half(r1, bit, sa.f[k][0], pa[j], pb[j], y0, y1, y2, y3);
        }
      }
    }
    // Higher spins come last, with strides that are multiples of the 256-index tile: their
    // digits are the same for the whole workgroup.  A missing partner (digit at the edge) gets
    // coefficient 0 and reads this thread's own index, so all loads of a batch of four nuclei
    // are in bounds and are issued together, each a unit-stride load.
    int64_t rem = (bx * kBlock) >> nh;
    for (int k0 = nh; k0 < sa.N; k0 += 4) {
      cx<R> pm0[4], pm1[4], pp0[4], pp1[4];
      R fm[4], fpl[4];
      bool r1v[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = k0 + j;
        fm[j] = R(0);
        fpl[j] = R(0);
        r1v[j] = true;
        if (k < sa.N) {
          const int dk = sa.d[k];
          const int64_t q = rem / dk;
          const int n = __builtin_amdgcn_readfirstlane((int)(rem - q * dk));
          rem = q;
          const int64_t st = sa.stride[k];
          const bool r1 = sa.rad[k] == 0;
          r1v[j] = r1;
          const R mk = R(0.5) * R(dk - 1) - R(n);
          if (r1) h1 += sa.a[k] * mk; else h2 += sa.a[k] * mk;
          const int64_t Pm = n > 0 ? M - st : M, Pp = n < dk - 1 ? M + st : M;
          fm[j] = n > 0 ? sa.f[k][n - 1] : R(0);
          fpl[j] = n < dk - 1 ? sa.f[k][n] : R(0);
          // minus partner (digit n-1) feeds the alpha components from beta ones; plus partner
          // (digit n+1) feeds beta components from alpha ones
          pm0[j] = X[(r1 ? 2 : 1) * Z + Pm];
          pm1[j] = X[3 * Z + Pm];
          pp0[j] = X[Pp];
          pp1[j] = X[(r1 ? 1 : 2) * Z + Pp];
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (k0 + j < sa.N) {
          if (r1v[j]) {
            y0 = cadd(y0, cscale(fm[j], pm0[j]));
            y1 = cadd(y1, cscale(fm[j], pm1[j]));
            y2 = cadd(y2, cscale(fpl[j], pp0[j]));
            y3 = cadd(y3, cscale(fpl[j], pp1[j]));
          } else {
            y0 = cadd(y0, cscale(fm[j], pm0[j]));
            y2 = cadd(y2, cscale(fm[j], pm1[j]));
            y1 = cadd(y1, cscale(fpl[j], pp0[j]));
            y3 = cadd(y3, cscale(fpl[j], pp1[j]));
          }
        }
      }
    }
    finish_term<R, MODE, NT>(ta, sa, fp, t, M, h1, h2, x0, x1, x2, x3, o0, o1, o2, o3, y0, y1, y2, y3);
    if (MODE == kFirst)
      nrm = (double)x0.x * x0.x + (double)x0.y * x0.y + (double)x1.x * x1.x + (double)x1.y * x1.y +
            (double)x2.x * x2.x + (double)x2.y * x2.y + (double)x3.x * x3.x + (double)x3.y * x3.y;
  }
  if (MODE == kFirst) {
    const double tot = block_sum(nrm, lds);
    if (tid == 0) ta.part_norm[L] = tot;
  }
}

// ---- complex-FP32 term kernel on index pairs
// Two consecutive complex FP32 numbers as one 16-byte vector.
using f4 = float __attribute__((ext_vector_type(4)));
template <bool ON>
__device__ __forceinline__ f4 ld4(const cx<float> *p) {
  const f4 *q = reinterpret_cast<const f4 *>(p);
  if constexpr (ON) return __builtin_nontemporal_load(q);
  else return *q;
}
template <bool ON>
__device__ __forceinline__ void st4(cx<float> *p, cx<float> a, cx<float> b) {
  f4 v;
  v.x = a.x;
  v.y = a.y;
  v.z = b.x;
  v.w = b.y;
  if constexpr (ON) __builtin_nontemporal_store(v, reinterpret_cast<f4 *>(p));
  else *reinterpret_cast<f4 *>(p) = v;
}
__device__ __forceinline__ cx<float> lo(f4 v) { return {v.x, v.y}; }
__device__ __forceinline__ cx<float> hi(f4 v) { return {v.z, v.w}; }

// H x accumulated for one nuclear index: the four components and the diagonal sums of the
// two radicals.
struct PairAcc {
  cx<float> y0, y1, y2, y3;
  float h1, h2;
};

// One spin-1/2 axis: the diagonal term a_k m_k and the flip-flop term from the partner's two
// components (p0, p1), with the radical chosen on values (no output chosen by a branch, so
// both PairAcc of a thread stay in registers).
__device__ __forceinline__ void pair_axis(PairAcc &A, bool r1, int bit, float a, float f, cx<float> p0,
                                          cx<float> p1) {
  const float am = a * (bit ? -0.5f : 0.5f);
  A.h1 += r1 ? am : 0.0f;
  A.h2 += r1 ? 0.0f : am;
  const cx<float> u0 = cscale(f, p0), u1 = cscale(f, p1), z = {0.0f, 0.0f};
  const cx<float> lo0 = csel(bit, u0, z), lo1 = csel(bit, u1, z), hi0 = csel(bit, z, u0), hi1 = csel(bit, z, u1);
  A.y0 = cadd(A.y0, lo0);
  A.y1 = cadd(A.y1, r1 ? lo1 : hi0);
  A.y2 = cadd(A.y2, r1 ? hi0 : lo1);
  A.y3 = cadd(A.y3, hi1);
}

// The two components of the partner that feed this index along a spin-1/2 axis: for the
// radical-1 electron, (aa, ab) or (ba, bb) of the partner; for radical 2, (aa, ba) or (ab, bb).
__device__ __forceinline__ int pair_c0(bool r1, int bit) { return r1 ? 2 * bit : bit; }
__device__ __forceinline__ int pair_c1(bool r1, int bit) { return r1 ? 2 * bit + 1 : bit + 2; }

// One Chebyshev term (complex FP32) with the same 256-index tile as k_cheb_tile, run by 128
// threads that own two consecutive indices M, M + 1 each.  Every global access is a 16-byte
// vector (two complex numbers), the partner along axis 0 is the thread's other index, the
// partners along axes 1..7 come from LDS (16-byte reads) and those along the slow axes from
// global memory; higher spins follow as in k_cheb_tile.  Needs at least 8 spin-1/2 nuclei
// first (Z a multiple of 256).
constexpr int kPairThreads = kBlock / 2;
constexpr int kPairBatch = 8;   // slow-axis partner pairs loaded together
template <int MODE, bool NT, bool Q>
__global__ __launch_bounds__(kPairThreads) void k_cheb_pair(TermArgs<float> ta, SysArgs<float> sa1) {
  __shared__ f4 tile[4 * kPairThreads];
  __shared__ double lds[2];
  const int64_t L = ta.remap ? xcd_remap(blockIdx.x, ta.tiles) : (int64_t)blockIdx.x;
  const TileRef t = tile_ref<Q>(ta, L, sa1.Z);
  const SysArgs<float> &sa = Q ? ta.systab[t.sys] : sa1;
  const int64_t bx = t.bx;
  const int tid = threadIdx.x;
  const int64_t M = bx * kBlock + 2 * tid;
  const int fi = t.fi;
  const FieldDev<float> fp = ta.fields[fi];
  const int64_t Z = t.Z;
  const cx<float> *X = ta.phin + t.vec;
  f4 xv[4], ov[4] = {};
  for (int e = 0; e < 4; ++e) xv[e] = ld4<false>(X + e * Z + M);
  if (MODE != kFirst) {
    const cx<float> *O = ta.phio + t.vec + M;
    for (int e = 0; e < 4; ++e) ov[e] = ld4<NT>(O + e * Z);
  }
  for (int e = 0; e < 4; ++e) tile[e * kPairThreads + tid] = xv[e];
  __syncthreads();
  const cx<float> zero = {0.0f, 0.0f};
  PairAcc A = {zero, zero, zero, zero, 0.0f, 0.0f}, B = A;   // index M, M + 1
  {  // axis 0: the other index of this thread
    const bool r1 = sa.rad[0] == 0;
    const float a = sa.a[0], f = sa.f[0][0];
    pair_axis(A, r1, 0, a, f, hi(xv[pair_c0(r1, 0)]), hi(xv[pair_c1(r1, 0)]));
    pair_axis(B, r1, 1, a, f, lo(xv[pair_c0(r1, 1)]), lo(xv[pair_c1(r1, 1)]));
  }
#pragma unroll
  for (int k = 1; k < 8; ++k) {   // axes 1..7: thread bit k-1, both indices share it
    const int bit = (tid >> (k - 1)) & 1;
    const int pt = tid ^ (1 << (k - 1));
    const bool r1 = sa.rad[k] == 0;
    const f4 q0 = tile[pair_c0(r1, bit) * kPairThreads + pt], q1 = tile[pair_c1(r1, bit) * kPairThreads + pt];
    pair_axis(A, r1, bit, sa.a[k], sa.f[k][0], lo(q0), lo(q1));
    pair_axis(B, r1, bit, sa.a[k], sa.f[k][0], hi(q0), hi(q1));
  }
  const int nh = sa.nhalf;
  for (int k0 = 8; k0 < nh; k0 += kPairBatch) {
    f4 pa[kPairBatch], pb[kPairBatch];
#pragma unroll
    for (int j = 0; j < kPairBatch; ++j) {
      const int k = k0 + j;
      if (k < nh) {
        const int bit = (int)((M >> k) & 1);
        const bool r1 = sa.rad[k] == 0;
        const int64_t P = M ^ ((int64_t)1 << k);
        pa[j] = ld4<false>(X + pair_c0(r1, bit) * Z + P);
        pb[j] = ld4<false>(X + pair_c1(r1, bit) * Z + P);
      }
    }
#pragma unroll
    for (int j = 0; j < kPairBatch; ++j) {
      const int k = k0 + j;
      if (k < nh) {
        const int bit = (int)((M >> k) & 1);
        const bool r1 = sa.rad[k] == 0;
        pair_axis(A, r1, bit, sa.a[k], sa.f[k][0], lo(pa[j]), lo(pb[j]));
        pair_axis(B, r1, bit, sa.a[k], sa.f[k][0], hi(pa[j]), hi(pb[j]));
      }
    }
  }
  // Higher spins: digits uniform over the workgroup (strides are multiples of 256); a missing
  // partner gets coefficient 0 and reads this thread's own pair.
  int64_t rem = (bx * kBlock) >> nh;
  for (int k0 = nh; k0 < sa.N; k0 += 2) {   // two nuclei per batch: eight 16-byte loads in flight
    f4 pm0[2], pm1[2], pp0[2], pp1[2];
    float fm[2], fpl[2];
    bool r1v[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int k = k0 + j;
      fm[j] = 0.0f;
      fpl[j] = 0.0f;
      r1v[j] = true;
      if (k < sa.N) {
        const int dk = sa.d[k];
        const int64_t q = rem / dk;
        const int n = __builtin_amdgcn_readfirstlane((int)(rem - q * dk));
        rem = q;
        const int64_t st = sa.stride[k];
        const bool r1 = sa.rad[k] == 0;
        r1v[j] = r1;
        const float am = sa.a[k] * (0.5f * (float)(dk - 1) - (float)n);
        A.h1 += r1 ? am : 0.0f;
        A.h2 += r1 ? 0.0f : am;
        B.h1 += r1 ? am : 0.0f;
        B.h2 += r1 ? 0.0f : am;
        const int64_t Pm = n > 0 ? M - st : M, Pp = n < dk - 1 ? M + st : M;
        fm[j] = n > 0 ? sa.f[k][n - 1] : 0.0f;
        fpl[j] = n < dk - 1 ? sa.f[k][n] : 0.0f;
        // minus partner (digit n-1) feeds the alpha components from beta ones; plus partner
        // (digit n+1) feeds beta components from alpha ones
        pm0[j] = ld4<false>(X + (r1 ? 2 : 1) * Z + Pm);
        pm1[j] = ld4<false>(X + 3 * Z + Pm);
        pp0[j] = ld4<false>(X + Pp);
        pp1[j] = ld4<false>(X + (r1 ? 1 : 2) * Z + Pp);
      }
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (k0 + j < sa.N) {
        const bool r1 = r1v[j];
        A.y0 = cadd(A.y0, cscale(fm[j], lo(pm0[j])));
        B.y0 = cadd(B.y0, cscale(fm[j], hi(pm0[j])));
        A.y3 = cadd(A.y3, cscale(fpl[j], lo(pp1[j])));
        B.y3 = cadd(B.y3, cscale(fpl[j], hi(pp1[j])));
        const cx<float> ua = cscale(fm[j], lo(pm1[j])), ub = cscale(fm[j], hi(pm1[j]));
        const cx<float> va = cscale(fpl[j], lo(pp0[j])), vb = cscale(fpl[j], hi(pp0[j]));
        A.y1 = cadd(A.y1, r1 ? ua : va);
        A.y2 = cadd(A.y2, r1 ? va : ua);
        B.y1 = cadd(B.y1, r1 ? ub : vb);
        B.y2 = cadd(B.y2, r1 ? vb : ub);
      }
    }
  }
  // phi_{n+1}, its singlet amplitude and the accumulator, two indices per 16-byte access
  cx<float> za[4], zb[4];
  term_z<float, MODE>(sa, fp, A.h1, A.h2, lo(xv[0]), lo(xv[1]), lo(xv[2]), lo(xv[3]), lo(ov[0]), lo(ov[1]),
                      lo(ov[2]), lo(ov[3]), A.y0, A.y1, A.y2, A.y3, za[0], za[1], za[2], za[3]);
  term_z<float, MODE>(sa, fp, B.h1, B.h2, hi(xv[0]), hi(xv[1]), hi(xv[2]), hi(xv[3]), hi(ov[0]), hi(ov[1]),
                      hi(ov[2]), hi(ov[3]), B.y0, B.y1, B.y2, B.y3, zb[0], zb[1], zb[2], zb[3]);
  const int64_t e0 = t.vec + M;
  cx<float> *O = ta.phio + e0;
  for (int e = 0; e < 4; ++e) st4<NT>(O + e * Z, za[e], zb[e]);
  st4<true>(ta.dnext + t.amp + M, csub(za[1], za[2]), csub(zb[1], zb[2]));
  const cx<float> *cf = ta.coef + (int64_t)fi * ta.n_terms;
  cx<float> *Ac = ta.acc + e0;
  if (MODE == kFirst) {
    const cx<float> a0 = cf[0], a1 = cf[1];
    for (int e = 0; e < 4; ++e)
      st4<NT>(Ac + e * Z, acc_value<float, MODE>(a0, a1, zero, zero, zero, lo(xv[e]), za[e]),
              acc_value<float, MODE>(a0, a1, zero, zero, zero, hi(xv[e]), zb[e]));
    st4<true>(ta.dfirst + t.amp + M, csub(lo(xv[1]), lo(xv[2])), csub(hi(xv[1]), hi(xv[2])));
  } else if (MODE == kAcc3) {
    const cx<float> am = cf[ta.n - 1], a0 = cf[ta.n], ap = cf[ta.n + 1];
    f4 v[4];
    for (int e = 0; e < 4; ++e) v[e] = ld4<NT>(Ac + e * Z);
    for (int e = 0; e < 4; ++e)
      st4<NT>(Ac + e * Z, acc_value<float, MODE>(am, a0, ap, lo(v[e]), lo(ov[e]), lo(xv[e]), za[e]),
              acc_value<float, MODE>(am, a0, ap, hi(v[e]), hi(ov[e]), hi(xv[e]), zb[e]));
  }
  if (MODE == kFirst) {
    double nrm = 0.0;
    for (int e = 0; e < 4; ++e)
      nrm += (double)xv[e].x * xv[e].x + (double)xv[e].y * xv[e].y + (double)xv[e].z * xv[e].z +
             (double)xv[e].w * xv[e].w;
    nrm = warp_sum(nrm);
    if ((tid & 63) == 0) lds[tid >> 6] = nrm;
    __syncthreads();
    if (tid == 0) ta.part_norm[L] = lds[0] + lds[1];
  }
}

// One Chebyshev term for any mix of spins (mixed-radix digits, partners from global memory).
template <typename R, int MODE, bool NT, bool Q>
__global__ __launch_bounds__(256) void k_cheb_gen(TermArgs<R> ta, SysArgs<R> sa1) {
  __shared__ double lds[4];
  const int64_t L = ta.remap ? xcd_remap(blockIdx.x, ta.tiles) : (int64_t)blockIdx.x;
  const TileRef t = tile_ref<Q>(ta, L, sa1.Z);
  const SysArgs<R> &sa = Q ? ta.systab[t.sys] : sa1;
  const int64_t M = t.bx * kBlock + threadIdx.x;
  const bool live = M < t.Z;
  const FieldDev<R> fp = ta.fields[t.fi];
  double nrm = 0.0;
  if (live) {
    const cx<R> zero = {R(0), R(0)};
    const int64_t Z = t.Z;
    const cx<R> *X = ta.phin + t.vec;
    cx<R> o0 = zero, o1 = zero, o2 = zero, o3 = zero;
    const cx<R> x0 = X[M], x1 = X[Z + M], x2 = X[2 * Z + M], x3 = X[3 * Z + M];
    if (MODE != kFirst) {
      const cx<R> *O = ta.phio + t.vec + M;
      o0 = ld_nt<NT>(O);
      o1 = ld_nt<NT>(O + Z);
      o2 = ld_nt<NT>(O + 2 * Z);
      o3 = ld_nt<NT>(O + 3 * Z);
    }
    cx<R> y0 = zero, y1 = zero, y2 = zero, y3 = zero;
    R h1 = R(0), h2 = R(0);
    int64_t rem = M;
    for (int k = 0; k < sa.N; ++k) {
      const int64_t st = sa.stride[k];
      const int dk = sa.d[k];
      const int64_t q = rem / dk;
      const int n = (int)(rem - q * dk);
      rem = q;
      const R mk = R(0.5) * R(dk - 1) - R(n);
      const bool r1 = sa.rad[k] == 0;
      if (r1) h1 += sa.a[k] * mk; else h2 += sa.a[k] * mk;
      if (n > 0) {        // partner digit n-1: beta component -> alpha component (I- S+)
        const R fk = sa.f[k][n - 1];
        const cx<R> *Pp = X + (M - st);
        if (r1) {
          y0 = cadd(y0, cscale(fk, Pp[2 * Z]));
          y1 = cadd(y1, cscale(fk, Pp[3 * Z]));
        } else {
          y0 = cadd(y0, cscale(fk, Pp[Z]));
          y2 = cadd(y2, cscale(fk, Pp[3 * Z]));
        }
      }
      if (n < dk - 1) {   // partner digit n+1: alpha component -> beta component (I+ S-)
        const R fk = sa.f[k][n];
        const cx<R> *Pp = X + (M + st);
        if (r1) {
          y2 = cadd(y2, cscale(fk, Pp[0]));
          y3 = cadd(y3, cscale(fk, Pp[Z]));
        } else {
          y1 = cadd(y1, cscale(fk, Pp[0]));
          y3 = cadd(y3, cscale(fk, Pp[2 * Z]));
        }
      }
    }
    finish_term<R, MODE, NT>(ta, sa, fp, t, M, h1, h2, x0, x1, x2, x3, o0, o1, o2, o3, y0, y1, y2, y3);
    if (MODE == kFirst)
      nrm = (double)x0.x * x0.x + (double)x0.y * x0.y + (double)x1.x * x1.x + (double)x1.y * x1.y +
            (double)x2.x * x2.x + (double)x2.y * x2.y + (double)x3.x * x3.x + (double)x3.y * x3.y;
  }
  if (MODE == kFirst) {
    const double tot = block_sum(nrm, lds);
    if (threadIdx.x == 0) ta.part_norm[L] = tot;
  }
}

// ----------------------------------------------------------------------------- in-step quadrature
// part[job][bx] = ( sum_M sum_r |sum_n ell_nr (-i)^n d_n(M)|^2 ,  sum_M |d_0(M)|^2 / 2 ).
// The factor ell is the same for every thread of a workgroup (one job, one field), so it
// is read through the scalar cache into SGPRs and used as the uniform FMA operand; each
// slab of singlet amplitudes is read once per pass of RC columns.
template <typename R>
using const_ptr = const __attribute__((address_space(4))) R *;

template <typename R, int RC, bool Q>
__global__ __launch_bounds__(256) void k_quad(QuadArgs<R> qa) {
  __shared__ double lds[4];
  const int64_t L = qa.remap ? xcd_remap(blockIdx.x, qa.tiles) : (int64_t)blockIdx.x;
  const TileRef t = tile_ref<Q>(qa, L, qa.Z);
  const int64_t M = t.bx * kBlock + threadIdx.x;
  const bool live = M < t.Z;
  const int fi = __builtin_amdgcn_readfirstlane(t.fi);
  const_ptr<R> ell = (const_ptr<R>)(qa.ell + (int64_t)fi * qa.n_terms * qa.rank_pad);
  const cx<R> *dp = qa.d + t.amp + (live ? M : 0);
  double acc = 0.0, ps = 0.0;
  if (live) {
    for (int r0 = 0; r0 < qa.rank_pad; r0 += RC) {
      cx<R> W[RC];
#pragma unroll
      for (int r = 0; r < RC; ++r) W[r] = {R(0), R(0)};
      cx<R> vn = ld_nt<true>(dp);
      for (int n = 0; n < qa.n_terms; ++n) {
        const cx<R> v = vn;
        if (n + 1 < qa.n_terms) vn = ld_nt<true>(dp + (int64_t)(n + 1) * qa.slab);
        cx<R> u;
        switch (n & 3) {          // multiply by (-i)^n
          case 0: u = v; break;
          case 1: u = {v.y, -v.x}; break;
          case 2: u = {-v.x, -v.y}; break;
          default: u = {-v.y, v.x}; break;
        }
        const_ptr<R> e = ell + (int64_t)n * qa.rank_pad + r0;
#pragma unroll
        for (int r = 0; r < RC; ++r) {
          const R l = e[r];
          W[r].x += l * u.x;
          W[r].y += l * u.y;
        }
      }
      R part = R(0);   // RC squares in the working precision, then accumulated in FP64
#pragma unroll
      for (int r = 0; r < RC; ++r) part += W[r].x * W[r].x + W[r].y * W[r].y;
      acc += (double)part;
    }
    const cx<R> v0 = dp[0];
    ps = 0.5 * ((double)v0.x * v0.x + (double)v0.y * v0.y);
  }
  const double s0 = block_sum(acc, lds);
  const double s1 = block_sum(ps, lds);
  if (threadIdx.x == 0) {
    qa.part[L * 2] = s0;
    qa.part[L * 2 + 1] = s1;
  }
}

// The same quadrature in complex FP32 on the matrix cores.  For the 256 nuclear indices of a
// tile, W = U ell with U[M][n] = (-i)^n d_n(M) is two real products: the real part of
// (-i)^n d_n is +x, +y, -x, -y of d_n = x + iy for n = 0, 1, 2, 3 (mod 4), the imaginary part
// +y, -x, -y, +x.  v_mfma_f32_16x16x4_f32 takes four terms per step, lane 16 g + i holding row
// i (a nuclear index) of term 4 k + g, so term mod 4 = g is fixed per lane and each lane picks
// and signs its component once per load.  Eight waves own two blocks of 16 rows each (32
// indices); a pass covers CB blocks of 16 columns, whose factor columns are staged in LDS with
// the row stride padded off multiples of 32 floats, so that the four term rows of a step fall
// in distinct banks.  Each wave loads the amplitudes of the next step while the matrix cores
// work on the current one; the other waves (seven per SIMD with three column blocks), each
// starting at its own eighth of the steps, hide the rest of the latency.  Only the sum of
// squares of W is kept, so the layout of the results does not matter.
using f32x4 = float __attribute__((ext_vector_type(4)));
constexpr int kQuadThreads = 512;
constexpr int kQuadWaves = kQuadThreads / 64;

__host__ __device__ constexpr int quad_lds_stride(int cb) { return 16 * cb + ((cb & 1) ? 0 : 16); }

template <int CB, bool Q>
__global__ __launch_bounds__(kQuadThreads) void k_quad_mx(QuadArgs<float> qa) {
  extern __shared__ float ls[];    // [4 nk][quad_lds_stride(CB)]
  __shared__ double red[2][kQuadWaves];
  constexpr int RC = 16 * CB, S = quad_lds_stride(CB);
  const int64_t L = qa.remap ? xcd_remap(blockIdx.x, qa.tiles) : (int64_t)blockIdx.x;
  const TileRef t = tile_ref<Q>(qa, L, qa.Z);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, i = lane & 15;
  const int fi = __builtin_amdgcn_readfirstlane(t.fi);
  const float *ell = qa.ell + (int64_t)fi * qa.n_terms * qa.rank_pad;
  const int nt = qa.n_terms, nk = (nt + 3) / 4;
  const bool swap = (g & 1) != 0;
  const float sre = (g & 2) ? -1.f : 1.f;
  const float sim = (g == 1 || g == 2) ? -1.f : 1.f;
  // rows M0 and M0 + 16 of the tile; a row beyond the job's Z reads as zero
  const int64_t M0 = t.bx * kBlock + wave * 32 + i;
  const bool live[2] = {M0 < t.Z, M0 + 16 < t.Z};
  const cx<float> *src = qa.d + t.amp + M0;
  auto load = [&](int k, cx<float> (&v)[2]) {
    const int n = 4 * k + g;
    const cx<float> *p = src + (int64_t)n * qa.slab;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
      v[rb] = (live[rb] && n < nt) ? ld_nt<true>(p + 16 * rb) : cx<float>{0.f, 0.f};
  };
  // Wave w starts at step w nk / 8 and wraps around, so that the waves of a workgroup, which
  // leave the staging barrier together, do not wait for memory in lockstep.
  const int k0 = wave * nk / kQuadWaves;
  double acc = 0.0;
  for (int r0 = 0; r0 < qa.rank_pad; r0 += RC) {
    cx<float> v[2];
    load(k0, v);
    __syncthreads();   // the previous pass has finished reading ls
    for (int e = threadIdx.x; e < 4 * nk * (RC / 4); e += kQuadThreads) {
      const int n = e / (RC / 4), c = 4 * (e - n * (RC / 4));
      f32x4 w = {0.f, 0.f, 0.f, 0.f};
      if (n < nt) w = *reinterpret_cast<const f32x4 *>(ell + (int64_t)n * qa.rank_pad + r0 + c);
      *reinterpret_cast<f32x4 *>(ls + n * S + c) = w;
    }
    __syncthreads();
    f32x4 cre[2][CB], cim[2][CB];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int c = 0; c < CB; ++c) cre[rb][c] = cim[rb][c] = f32x4{0.f, 0.f, 0.f, 0.f};
    int k = k0;
    for (int kk = 0; kk < nk; ++kk) {
      float b[CB];
#pragma unroll
      for (int c = 0; c < CB; ++c) b[c] = ls[(4 * k + g) * S + 16 * c + i];
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) {
        const float are = sre * (swap ? v[rb].y : v[rb].x);
        const float aim = sim * (swap ? v[rb].x : v[rb].y);
#pragma unroll
        for (int c = 0; c < CB; ++c) {
          cre[rb][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(are, b[c], cre[rb][c], 0, 0, 0);
          cim[rb][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(aim, b[c], cim[rb][c], 0, 0, 0);
        }
      }
      k = k + 1 == nk ? 0 : k + 1;
      if (kk + 1 < nk) load(k, v);
    }
    float part = 0.f;   // squares in FP32 per pass, then accumulated in FP64
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int c = 0; c < CB; ++c)
#pragma unroll
        for (int e = 0; e < 4; ++e) part += cre[rb][c][e] * cre[rb][c][e] + cim[rb][c][e] * cim[rb][c][e];
    acc += (double)part;
  }
  double ps = 0.0;   // |d_0|^2 / 2 of each row, from the lanes of term 0
  if (g == 0) {
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
      if (live[rb]) {
        const cx<float> v0 = src[16 * rb];
        ps += 0.5 * ((double)v0.x * v0.x + (double)v0.y * v0.y);
      }
  }
  acc = warp_sum(acc);
  ps = warp_sum(ps);
  if (lane == 0) {
    red[0][wave] = acc;
    red[1][wave] = ps;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s0 = 0.0, s1 = 0.0;
    for (int w = 0; w < kQuadWaves; ++w) {
      s0 += red[0][w];
      s1 += red[1][w];
    }
    qa.part[L * 2] = s0;
    qa.part[L * 2 + 1] = s1;
  }
}

// Dynamic LDS of k_quad_mx for a pass of cb column blocks; 0 when it exceeds the 64 KB a
// launch gets without a raised limit (the VALU kernel runs instead).
static int64_t quad_mx_lds(int n_terms, int cb) {
  const int64_t b = (int64_t)4 * ((n_terms + 3) / 4) * quad_lds_stride(cb) * (int64_t)sizeof(float);
  return b <= 65536 ? b : 0;
}

// Term kernel variants: any mix of spins, the 256-index tile, and the tile on index pairs.
enum TermKernel { kTermGen = 0, kTermTile = 1, kTermPair = 2 };

template <typename R, int MODE, bool NT, bool Q>
static void launch_term_q(int kind, unsigned grid, hipStream_t st, const TermArgs<R> &ta, const SysArgs<R> &sa) {
  if constexpr (std::is_same<R, float>::value) {
    if (kind == kTermPair) {
      hipLaunchKernelGGL((k_cheb_pair<MODE, NT, Q>), dim3(grid), dim3(kPairThreads), 0, st, ta, sa);
      return;
    }
  }
  if (kind == kTermGen)
    hipLaunchKernelGGL((k_cheb_gen<R, MODE, NT, Q>), dim3(grid), dim3(kBlock), 0, st, ta, sa);
  else
    hipLaunchKernelGGL((k_cheb_tile<R, MODE, NT, Q>), dim3(grid), dim3(kBlock), 0, st, ta, sa);
}

template <typename R, int MODE, bool NT>
static void launch_term_t(int kind, bool q, unsigned grid, hipStream_t st, const TermArgs<R> &ta,
                          const SysArgs<R> &sa) {
  if (q) launch_term_q<R, MODE, NT, true>(kind, grid, st, ta, sa);
  else launch_term_q<R, MODE, NT, false>(kind, grid, st, ta, sa);
}

// q: the launch spans the job queue of several systems (per-job descriptors) rather than the
// jobs of one system.
template <typename R>
static void launch_term(int mode, int kind, bool nt, bool q, unsigned grid, hipStream_t st, const TermArgs<R> &ta,
                        const SysArgs<R> &sa) {
  switch (mode * 2 + (nt ? 1 : 0)) {
    case kFirst * 2: launch_term_t<R, kFirst, false>(kind, q, grid, st, ta, sa); break;
    case kFirst * 2 + 1: launch_term_t<R, kFirst, true>(kind, q, grid, st, ta, sa); break;
    case kPlain * 2: launch_term_t<R, kPlain, false>(kind, q, grid, st, ta, sa); break;
    case kPlain * 2 + 1: launch_term_t<R, kPlain, true>(kind, q, grid, st, ta, sa); break;
    case kAcc3 * 2: launch_term_t<R, kAcc3, false>(kind, q, grid, st, ta, sa); break;
    default: launch_term_t<R, kAcc3, true>(kind, q, grid, st, ta, sa); break;
  }
}

template <typename R, bool Q>
static void launch_quad_q(int rcw, unsigned grid, hipStream_t st, const QuadArgs<R> &qa) {
  switch (rcw) {
    case 64: hipLaunchKernelGGL((k_quad<R, 64, Q>), dim3(grid), dim3(kBlock), 0, st, qa); break;
    case 56: hipLaunchKernelGGL((k_quad<R, 56, Q>), dim3(grid), dim3(kBlock), 0, st, qa); break;
    case 48: hipLaunchKernelGGL((k_quad<R, 48, Q>), dim3(grid), dim3(kBlock), 0, st, qa); break;
    case 40: hipLaunchKernelGGL((k_quad<R, 40, Q>), dim3(grid), dim3(kBlock), 0, st, qa); break;
    case 32: hipLaunchKernelGGL((k_quad<R, 32, Q>), dim3(grid), dim3(kBlock), 0, st, qa); break;
    case 24: hipLaunchKernelGGL((k_quad<R, 24, Q>), dim3(grid), dim3(kBlock), 0, st, qa); break;
    case 16: hipLaunchKernelGGL((k_quad<R, 16, Q>), dim3(grid), dim3(kBlock), 0, st, qa); break;
    default: hipLaunchKernelGGL((k_quad<R, 8, Q>), dim3(grid), dim3(kBlock), 0, st, qa); break;
  }
}

template <bool Q>
static void launch_quad_mx(int cb, unsigned grid, size_t lds, hipStream_t st, const QuadArgs<float> &qa) {
  switch (cb) {
    case 4: hipLaunchKernelGGL((k_quad_mx<4, Q>), dim3(grid), dim3(kQuadThreads), lds, st, qa); break;
    case 3: hipLaunchKernelGGL((k_quad_mx<3, Q>), dim3(grid), dim3(kQuadThreads), lds, st, qa); break;
    case 2: hipLaunchKernelGGL((k_quad_mx<2, Q>), dim3(grid), dim3(kQuadThreads), lds, st, qa); break;
    default: hipLaunchKernelGGL((k_quad_mx<1, Q>), dim3(grid), dim3(kQuadThreads), lds, st, qa); break;
  }
}

// Complex FP32 passes of a multiple of 16 columns run on the matrix cores (unless the
// staged factor would not fit the LDS); everything else on the vector ALUs.
template <typename R>
static void launch_quad(int rcw, bool q, unsigned grid, hipStream_t st, const QuadArgs<R> &qa) {
  if constexpr (std::is_same<R, float>::value) {
    const int64_t lds = rcw % 16 == 0 ? quad_mx_lds(qa.n_terms, rcw / 16) : 0;
    if (lds > 0) {
      if (q) launch_quad_mx<true>(rcw / 16, grid, (size_t)lds, st, qa);
      else launch_quad_mx<false>(rcw / 16, grid, (size_t)lds, st, qa);
      return;
    }
  }
  if (q) launch_quad_q<R, true>(rcw, grid, st, qa);
  else launch_quad_q<R, false>(rcw, grid, st, qa);
}

// ----------------------------------------------------------------------------- LDS-resident propagation
// Sum over a workgroup of up to 1024 threads (every thread must call it).
__device__ __forceinline__ double block_sum_any(double v, double *lds) {
  v = warp_sum(v);
  const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  if ((threadIdx.x & 63) == 0) lds[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < nw; ++i) t += lds[i];
  __syncthreads();
  return t;
}

// One workgroup propagates one wavepacket for all of its steps.  Thread M owns nuclear index M:
// its four components of phi_n and phi_{n-1}, of the step accumulator and its kResRank
// quadrature sums stay in registers; the components of phi_n are exchanged with the partners
// through a ping-pong LDS buffer, one barrier per term.
template <typename R, int MAXB, int RK>
__global__ __launch_bounds__(MAXB) void k_resident(ResArgs<R> ra) {
  extern __shared__ unsigned char smem_raw[];
  cx<R> *buf = reinterpret_cast<cx<R> *>(smem_raw);   // [2][4][Zb]
  __shared__ double lds[16];
  const int Zb = blockDim.x;
  const ResJob jb = ra.jobs[blockIdx.x];
  const int si = __builtin_amdgcn_readfirstlane(jb.sys);
  const int fi = __builtin_amdgcn_readfirstlane(jb.field);
  const SysArgs<R> &sa = ra.sys[si].sa;
  const ResField<R> F = ra.fields[fi];
  const FieldDev<R> fp = F.fd;
  const int64_t Z = sa.Z;
  const int M = threadIdx.x;
  const bool live = M < Z;
  const cx<R> zero = {R(0), R(0)};
  const_ptr<R> ell = (const_ptr<R>)(ra.ell + F.ell_off);
  const cx<R> *cf = ra.coef + F.coef_off;
  const int N = sa.N;

  // initial wavepacket |S> (x) prod_k |Omega_k>
  cx<R> x0 = zero, x1 = zero, x2 = zero, x3 = zero;
  if (live) {
    const cx<double> *t = ra.tab + ra.sys[si].tab_off + (int64_t)jb.sample * N * (RP_MAX_TWO_I + 1);
    cx<double> p = {M_SQRT1_2, 0.0};
    int rem = M;
    for (int k = 0; k < N; ++k) {
      const int n = rem % sa.d[k];
      rem /= sa.d[k];
      const cx<double> c = t[k * (RP_MAX_TWO_I + 1) + n];
      p = {p.x * c.x - p.y * c.y, p.x * c.y + p.y * c.x};
    }
    x1 = {R(p.x), R(p.y)};
    x2 = {R(-p.x), R(-p.y)};
  }
  const double kS = ra.sys[si].kS, kmin = ra.sys[si].kmin, rtol = ra.sys[si].rtol;
  double phi = 0.0, prev = 1.0 + 1e-6;
  bool bad = false;
  for (int step = 0; step < F.n_steps; ++step) {
    // norm at the step start, and the wavepacket into buffer 0
    double nrm = 0.0;
    if (live) {
      buf[M] = x0;
      buf[Zb + M] = x1;
      buf[2 * Zb + M] = x2;
      buf[3 * Zb + M] = x3;
      nrm = (double)x0.x * x0.x + (double)x0.y * x0.y + (double)x1.x * x1.x + (double)x1.y * x1.y +
            (double)x2.x * x2.x + (double)x2.y * x2.y + (double)x3.x * x3.x + (double)x3.y * x3.y;
    }
    nrm = block_sum_any(nrm, lds);   // also orders the buffer writes before the first term
    const double decay = exp(-kmin * step * F.dt);
    if (!(decay * nrm <= prev * (1.0 + rtol) + 1e-300)) bad = true;
    prev = decay * nrm;
    cx<R> W[RK];
#pragma unroll
    for (int r = 0; r < RK; ++r) W[r] = zero;
    cx<R> a0v = zero, a1v = zero, a2v = zero, a3v = zero;   // step accumulator
    cx<R> o0 = zero, o1 = zero, o2 = zero, o3 = zero;       // phi_{n-1}
    if (live) {   // term 0 contributes a_0 phi_0 and its singlet amplitude
      const cx<R> c0 = cf[0];
      a0v = cmul(c0, x0);
      a1v = cmul(c0, x1);
      a2v = cmul(c0, x2);
      a3v = cmul(c0, x3);
      const cx<R> d = csub(x1, x2);
#pragma unroll
      for (int r = 0; r < RK; ++r) {
        const R l = ell[r];
        W[r].x += l * d.x;
        W[r].y += l * d.y;
      }
    }
    for (int n = 0; n + 1 < F.n_terms; ++n) {
      const cx<R> *cur = buf + (n & 1) * 4 * Zb;
      cx<R> *nxt = buf + ((n + 1) & 1) * 4 * Zb;
      if (live) {
        cx<R> y0 = zero, y1 = zero, y2 = zero, y3 = zero;
        R h1 = R(0), h2 = R(0);
        int rem = M;
        for (int k = 0; k < N; ++k) {
          const int dk = sa.d[k], st = sa.stride[k];
          const int nd = rem % dk;
          rem /= dk;
          const R mk = R(0.5) * R(dk - 1) - R(nd);
          const bool r1 = sa.rad[k] == 0;
          if (r1) h1 += sa.a[k] * mk; else h2 += sa.a[k] * mk;
          if (nd > 0) {        // partner digit n-1: beta component -> alpha component
            const R f = sa.f[k][nd - 1];
            const int P = M - st;
            if (r1) {
              y0 = cadd(y0, cscale(f, cur[2 * Zb + P]));
              y1 = cadd(y1, cscale(f, cur[3 * Zb + P]));
            } else {
              y0 = cadd(y0, cscale(f, cur[Zb + P]));
              y2 = cadd(y2, cscale(f, cur[3 * Zb + P]));
            }
          }
          if (nd < dk - 1) {   // partner digit n+1: alpha component -> beta component
            const R f = sa.f[k][nd];
            const int P = M + st;
            if (r1) {
              y2 = cadd(y2, cscale(f, cur[P]));
              y3 = cadd(y3, cscale(f, cur[Zb + P]));
            } else {
              y1 = cadd(y1, cscale(f, cur[P]));
              y3 = cadd(y3, cscale(f, cur[2 * Zb + P]));
            }
          }
        }
        const R hs = R(0.5) * (h1 + h2), hd = R(0.5) * (h1 - h2), hj = R(0.5) * sa.J;
        y0 = cadd(y0, cscale(fp.omega + hs + hj, x0));
        y1 = cadd(y1, cadd(cscale(hd - hj, x1), cscale(sa.J, x2)));
        y2 = cadd(y2, cadd(cscale(-hd - hj, x2), cscale(sa.J, x1)));
        y3 = cadd(y3, cscale(-fp.omega - hs + hj, x3));
        const cx<R> tt = {R(0.5) * (x1.x - x2.x), R(0.5) * (x1.y - x2.y)};
        const cx<R> ibt = {-sa.beta * tt.y, sa.beta * tt.x};
        y1 = cadd(y1, ibt);
        y2 = csub(y2, ibt);
        const cx<R> c = {fp.c_re, fp.c_im};
        const R s = n == 0 ? fp.s1 : fp.s2;
        cx<R> z0 = cscale(s, csub(y0, cmul(c, x0)));
        cx<R> z1 = cscale(s, csub(y1, cmul(c, x1)));
        cx<R> z2 = cscale(s, csub(y2, cmul(c, x2)));
        cx<R> z3 = cscale(s, csub(y3, cmul(c, x3)));
        if (n > 0) {
          z0 = csub(z0, o0);
          z1 = csub(z1, o1);
          z2 = csub(z2, o2);
          z3 = csub(z3, o3);
        }
        nxt[M] = z0;
        nxt[Zb + M] = z1;
        nxt[2 * Zb + M] = z2;
        nxt[3 * Zb + M] = z3;
        const cx<R> an = cf[n + 1];
        a0v = cadd(a0v, cmul(an, z0));
        a1v = cadd(a1v, cmul(an, z1));
        a2v = cadd(a2v, cmul(an, z2));
        a3v = cadd(a3v, cmul(an, z3));
        const cx<R> v = csub(z1, z2);
        cx<R> u;
        switch ((n + 1) & 3) {    // multiply by (-i)^(n+1)
          case 0: u = v; break;
          case 1: u = {v.y, -v.x}; break;
          case 2: u = {-v.x, -v.y}; break;
          default: u = {-v.y, v.x}; break;
        }
        const_ptr<R> e = ell + (int64_t)(n + 1) * kResRank;
#pragma unroll
        for (int r = 0; r < RK; ++r) {
          const R l = e[r];
          W[r].x += l * u.x;
          W[r].y += l * u.y;
        }
        o0 = x0;
        o1 = x1;
        o2 = x2;
        o3 = x3;
        x0 = z0;
        x1 = z1;
        x2 = z2;
        x3 = z3;
      }
      __syncthreads();
    }
    R part = R(0);
#pragma unroll
    for (int r = 0; r < RK; ++r) part += W[r].x * W[r].x + W[r].y * W[r].y;
    const double y = block_sum_any(live ? (double)part : 0.0, lds);
    phi += kS * decay * y;
    if (!(y == y)) bad = true;
    x0 = a0v;
    x1 = a1v;
    x2 = a2v;
    x3 = a3v;
  }
  if (threadIdx.x == 0) {
    ra.phi[jb.out] = phi;
    if (bad) atomicOr(ra.flag, 1);
  }
}

// ----------------------------------------------------------------------------- per-step finalisation
// One workgroup per job: sums the per-workgroup partials of the quadrature and of the norm.
__global__ __launch_bounds__(256) void k_finalize(FinArgs fa) {
  __shared__ double lds[4];
  const int64_t job = fa.slots ? fa.slots[blockIdx.x] : blockIdx.x;
  int64_t b0 = job * fa.nbx, nb = fa.nbx;
  int fi;
  double kS = fa.kS, kmin = fa.kmin;
  if (fa.jobs) {   // job queue: the job's own tiles and rates
    const QJob &j = fa.jobs[job];
    b0 = j.blk;
    nb = j.nbx;
    fi = j.field;
    kS = fa.sys_k[2 * j.sys];
    kmin = fa.sys_k[2 * j.sys + 1];
  } else {
    fi = fa.job_field[job];
  }
  double y = 0.0, nrm = 0.0, ps = 0.0;
  for (int64_t b = threadIdx.x; b < nb; b += kBlock) {
    y += fa.part_q[(b0 + b) * 2];
    nrm += fa.part_norm[b0 + b];
    if (fa.ps_t) ps += fa.part_q[(b0 + b) * 2 + 1];
  }
  y = block_sum(y, lds);
  nrm = block_sum(nrm, lds);
  if (fa.ps_t) ps = block_sum(ps, lds);
  if (threadIdx.x != 0) return;
  const int32_t step = fa.stepc[job];
  fa.stepc[job] = step + 1;
  const double decay = exp(-kmin * step * fa.dt[fi]);
  fa.phi[job] += kS * decay * y;
  if (fa.ps_t && step < fa.ps_len) fa.ps_t[fa.dst[job] * fa.ps_len + step] = decay * ps;
  const double Nt = decay * nrm;           // population N(t_j) of the wavepacket
  if (!(Nt <= fa.prev_norm[job] * (1.0 + fa.rtol) + 1e-300) || !(y == y)) atomicOr(fa.flag, 1);
  fa.prev_norm[job] = Nt;
}

// Job queue: clears the sums of the slots that take new jobs.
__global__ __launch_bounds__(256) void k_slots_reset(const int32_t *slots, int64_t n, double *phi, double *prev,
                                                     int32_t *stepc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t s = slots[i];
  phi[s] = 0.0;
  prev[s] = 1.0 + 1e-6;
  stepc[s] = 0;
}

// Job queue: writes the yields of the slots whose jobs have done their steps.
__global__ __launch_bounds__(256) void k_slots_scatter(const int32_t *slots, int64_t n, const double *phi,
                                                       const int64_t *dst, double *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t s = slots[i];
  out[dst[s]] = phi[s];
}

__global__ __launch_bounds__(256) void k_fill(double *p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ __launch_bounds__(256) void k_scatter(const double *src, const int64_t *dst_idx, double *dst,
                                                 int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[dst_idx[i]] = src[i];
}

// ----------------------------------------------------------------------------- statistics (Eq. 23)
struct StatArgs {
  const double *phi, *g, *mu, *beta, *mu_err;
  double *mean, *err;
  int64_t M;
};

__global__ __launch_bounds__(256) void k_stats(StatArgs a) {
  __shared__ double lds[4];
  const int b = blockIdx.x;
  const double *p = a.phi + (int64_t)b * a.M;
  const double *g = a.g ? a.g + (int64_t)b * a.M : nullptr;
  const double be = a.g ? a.beta[b] : 0.0, mu = a.g ? a.mu[b] : 0.0;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < a.M; i += blockDim.x) s += g ? p[i] - be * (g[i] - mu) : p[i];
  const double tot = block_sum(s, lds);
  __shared__ double mean_s;
  if (threadIdx.x == 0) mean_s = tot / (double)a.M;
  __syncthreads();
  const double m = mean_s;
  double q = 0.0;
  for (int64_t i = threadIdx.x; i < a.M; i += blockDim.x) {
    const double v = (g ? p[i] - be * (g[i] - mu) : p[i]) - m;
    q += v * v;
  }
  const double qt = block_sum(q, lds);
  if (threadIdx.x == 0) {
    a.mean[b] = m;
    const double e2 = a.M > 1 ? qt / (double)(a.M - 1) / (double)a.M : 0.0;
    a.err[b] = sqrt(e2 + (a.g && a.mu_err ? be * be * a.mu_err[b] * a.mu_err[b] : 0.0));
  }
}

// Inverse-variance combination of two independent unbiased estimates per field.
__global__ __launch_bounds__(256) void k_combine(const double *ma, const double *ea, const double *mb,
                                                 const double *eb, int32_t nB, double *mean, double *err) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nB) return;
  const double va = ea[b] * ea[b], vb = eb[b] * eb[b];
  if (va == 0.0 || vb == 0.0) {   // an exact estimate wins outright
    const bool a_exact = va == 0.0;
    mean[b] = a_exact ? ma[b] : mb[b];
    err[b] = 0.0;
    return;
  }
  const double wa = 1.0 / va, wb = 1.0 / vb;
  mean[b] = (wa * ma[b] + wb * mb[b]) / (wa + wb);
  err[b] = 1.0 / sqrt(wa + wb);
}

// Per-field beta = Cov(phi, g) / Var(g) (two passes: means, then centred sums).
struct BetaArgs {
  const double *phi, *g;
  double *beta;
  int64_t M;
};

__global__ __launch_bounds__(256) void k_beta(BetaArgs a) {
  __shared__ double lds[4];
  __shared__ double means[2];
  const double *p = a.phi + (int64_t)blockIdx.x * a.M, *g = a.g + (int64_t)blockIdx.x * a.M;
  double sp = 0.0, sg = 0.0;
  for (int64_t i = threadIdx.x; i < a.M; i += blockDim.x) {
    sp += p[i];
    sg += g[i];
  }
  const double tp = block_sum(sp, lds), tg = block_sum(sg, lds);
  if (threadIdx.x == 0) {
    means[0] = tp / (double)a.M;
    means[1] = tg / (double)a.M;
  }
  __syncthreads();
  double c = 0.0, v = 0.0;
  for (int64_t i = threadIdx.x; i < a.M; i += blockDim.x) {
    const double dp = p[i] - means[0], dg = g[i] - means[1];
    c += dp * dg;
    v += dg * dg;
  }
  const double tc = block_sum(c, lds), tv = block_sum(v, lds);
  if (threadIdx.x == 0) a.beta[blockIdx.x] = tv > 0.0 ? tc / tv : 0.0;
}

// ============================================================================= host side
static thread_local std::string g_err;

static int fail(int code, const std::string &m) {
  g_err = m;
  return code;
}

int mlp_fail(int code, const char *msg) { return fail(code, msg); }

#define HIPCHK(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) return fail(RP_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

static int validate_system(const rp_system *s) {
  if (!s) return fail(RP_EINVAL, "null system");
  const int N1 = s->n_nuc[0], N2 = s->n_nuc[1];
  if (N1 < 0 || N2 < 0 || N1 + N2 > RP_MAX_NUCLEI) return fail(RP_EINVAL, "nucleus counts out of range");
  if (N1 + N2 > 0 && (!s->two_I || !s->a_mT)) return fail(RP_EINVAL, "null two_I or a_mT");
  double Z = 1.0;
  for (int k = 0; k < N1 + N2; ++k) {
    if (s->two_I[k] < 1 || s->two_I[k] > RP_MAX_TWO_I) return fail(RP_EINVAL, "two_I out of range 1..4");
    if (!std::isfinite(s->a_mT[k])) return fail(RP_EINVAL, "non-finite hyperfine constant");
    Z *= s->two_I[k] + 1;
  }
  if (Z > 2147483647.0 / 4) return fail(RP_EINVAL, "nuclear Hilbert space too large");
  if (!(s->kS >= 0.0) || !(s->kT >= 0.0) || !std::isfinite(s->kS) || !std::isfinite(s->kT))
    return fail(RP_EINVAL, "rate constants must be finite and >= 0");
  if (!(s->T_us > 0.0) || !std::isfinite(s->T_us)) return fail(RP_EINVAL, "T must be > 0");
  if (!std::isfinite(s->J_mT)) return fail(RP_EINVAL, "non-finite J");
  if (s->gamma < 0.0 || !std::isfinite(s->gamma)) return fail(RP_EINVAL, "gamma must be >= 0");
  return RP_OK;
}

struct Profile {
  double term_ms = 0, term_launches = 0, elems = 0, bytes = 0, quad_ms = 0, quad_launches = 0,
         total_ms = 0, terms = 0;
};
static thread_local Profile g_prof;

// Event pairs around groups of launches, resolved after the stream is synchronised.
struct EventLog {
  bool on = false;
  std::vector<hipEvent_t> ev;
  std::vector<int> kind;   // 0: term kernels, 1: quadrature
  hipEvent_t mark(hipStream_t st) {
    hipEvent_t e = nullptr;
    if (!on) return e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    (void)hipEventRecord(e, st);
    ev.push_back(e);
    return e;
  }
  void close(int k) { if (on) kind.push_back(k); }
  void resolve(Profile &p) {
    for (size_t i = 0; i + 1 < ev.size(); i += 2) {
      float ms = 0.f;
      if (ev[i] && ev[i + 1] && hipEventElapsedTime(&ms, ev[i], ev[i + 1]) == hipSuccess) {
        if (kind[i / 2] == 0) p.term_ms += ms; else p.quad_ms += ms;
      }
    }
  }
  ~EventLog() { for (auto e : ev) if (e) (void)hipEventDestroy(e); }
};

static double gamma_of(const rp_system *s) { return s->gamma > 0.0 ? s->gamma : 176.085963023; }

struct Opts {
  int precision = 64, init_mode = 0, flags = 0, krylov = 16;
  double tol = 0, rdt = 0, r_scale = 1.0, chol_tol = 0, max_growth = 0;
  bool tol_set = false;
  int64_t workspace = 0;
  int64_t ps_len = 0;
};

static int read_opts(const rp_opts *o, Opts &out) {
  out = Opts();
  if (o) {
    if (o->precision != 0 && o->precision != 32 && o->precision != 64)
      return fail(RP_EINVAL, "precision must be 32 or 64");
    if (o->precision) out.precision = o->precision;
    if (o->init_mode != 0 && o->init_mode != 1) return fail(RP_EINVAL, "init_mode must be 0 or 1");
    out.init_mode = o->init_mode;
    if (o->tol < 0 || o->rdt < 0 || o->r_scale < 0 || o->workspace_bytes < 0 || o->max_growth < 0)
      return fail(RP_EINVAL, "negative option");
    if (o->max_growth != 0 && !(o->max_growth >= 2.0)) return fail(RP_EINVAL, "max_growth must be >= 2");
    const int known =
        RP_FLAG_PROFILE | RP_FLAG_TILED | RP_FLAG_XCD_LOCAL | RP_FLAG_XCD_SPREAD | RP_FLAG_NO_GRAPH | RP_FLAG_ARNOLDI |
        RP_FLAG_TERM_SCALAR | RP_FLAG_AXES_HIGH_FIRST;
    if ((o->flags & ~known) != 0) return fail(RP_EINVAL, "unknown flags");
    if (o->krylov_dim != 0 && (o->krylov_dim < 2 || o->krylov_dim > 32))
      return fail(RP_EINVAL, "krylov_dim must be 0 or in [2, 32]");
    if (o->krylov_dim) out.krylov = o->krylov_dim;
    out.flags = o->flags;
    out.tol_set = o->tol > 0;
    if (o->tol > 0) out.tol = o->tol;
    if (o->rdt > 0) out.rdt = o->rdt;
    if (o->r_scale > 0) out.r_scale = o->r_scale;
    out.workspace = o->workspace_bytes;
    out.max_growth = o->max_growth;
    if (o->ps_t_len < 0) return fail(RP_EINVAL, "negative ps_t_len");
    out.ps_len = o->ps_t_len;
  }
  if (out.tol == 0) out.tol = out.precision == 64 ? 1e-14 : 1e-9;
  out.chol_tol = out.precision == 64 ? 1e-17 : 1e-12;
  // The worst case assumes an eigenvector at a corner of the dissipative strip carrying the
  // whole wavepacket; wavepackets with a singlet electron state carry little weight there, and
  // measured errors stay at the rounding level far beyond eps * growth = tolerance.
  if (out.max_growth == 0) out.max_growth = out.precision == 64 ? 1e10 : 1e6;
  // Default step: the series needs about r*dt + O((r*dt)^(1/3)) terms and the quadrature rank
  // grows like r*dt/pi; measured on the 7+7 sweep, r*dt = 100 is the sweet spot for complex
  // FP32 and within 1 % of the best for FP64.
  if (out.rdt == 0) out.rdt = 100.0;
  if (out.rdt > 4000) return fail(RP_EINVAL, "rdt too large");
  return RP_OK;
}

template <typename R>
static SysArgs<R> make_sysargs(const SystemSpec &s) {
  SysArgs<R> a;
  std::memset(&a, 0, sizeof(a));
  a.N = s.N();
  a.N1 = s.N1;
  a.Z = s.Z;
  a.J = (R)s.J;
  // i beta P_S reproduces -i (dk/2) P_x together with the shift (see plan.hpp).
  a.beta = (R)(s.kS >= s.kT ? -0.5 * (s.kS - s.kT) : 0.5 * (s.kT - s.kS));
  a.all_half = 1;
  a.nhalf = 0;
  while (a.nhalf < a.N && s.two_I[a.nhalf] == 1) ++a.nhalf;
  a.tiled = (a.nhalf == a.N || a.nhalf >= 8) ? 1 : 0;
  int64_t st = 1;
  for (int k = 0; k < a.N; ++k) {
    a.stride[k] = (int32_t)st;
    a.d[k] = s.two_I[k] + 1;
    a.rad[k] = s.rad[k];
    if (s.two_I[k] != 1) a.all_half = 0;
    int sh = 0;
    while ((int64_t(1) << sh) < st) ++sh;
    a.shift[k] = sh;
    a.a[k] = (R)s.a[k];
    const double I = 0.5 * s.two_I[k];
    for (int n = 0; n < s.two_I[k]; ++n) {
      const double m = I - n;   // link between m and m-1
      a.f[k][n] = (R)(0.5 * s.a[k] * std::sqrt(I * (I + 1.0) - m * (m - 1.0)));
    }
    st *= a.d[k];
  }
  return a;
}

static unsigned grid1(int64_t n) { return (unsigned)((n + 255) / 256); }

// Device workspace of one call, carved from one block: the block rp_propagate allocates for
// the call on its stream, or the library's static scratch area (rp_propagate_static).  Every
// piece is 256-byte aligned; Sizer counts the same rounding, so a layout measured with Sizer
// fits an Arena of that many bytes exactly.
static int64_t round256(int64_t bytes) { return (std::max<int64_t>(bytes, 1) + 255) & ~int64_t(255); }
struct Sizer {
  int64_t used = 0;
  template <typename T>
  void add(int64_t n) { used += round256(n * (int64_t)sizeof(T)); }
};
struct Arena {
  char *base = nullptr;
  int64_t cap = 0, used = 0;
  bool overflow = false;
  template <typename T>
  T *take(int64_t n) {
    const int64_t b = round256(n * (int64_t)sizeof(T));
    if (used + b > cap) {
      overflow = true;
      return nullptr;
    }
    T *p = reinterpret_cast<T *>(base + used);
    used += b;
    return p;
  }
};

__global__ __launch_bounds__(256) void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Plans every (system, field) pair of a call on host threads.
static int plan_many(const std::vector<const SystemSpec *> &specs, const std::vector<const double *> &B, int nB,
                     const Opts &op, std::vector<FieldPlan> &plans) {
  const int tot = (int)specs.size() * nB;
  plans.assign(tot, FieldPlan());
  std::vector<std::string> msgs(tot);
  std::vector<char> ok(tot, 0);
  const int nth = std::max(1, std::min<int>(tot, (int)std::thread::hardware_concurrency()));
  std::vector<std::thread> th;
  for (int t = 0; t < nth; ++t)
    th.emplace_back([&, t]() {
      for (int q = t; q < tot; q += nth)
        ok[q] = plan_field(*specs[q / nB], B[q / nB][q % nB], op.tol, op.rdt, op.r_scale, op.chol_tol, op.max_growth,
                           plans[q], msgs[q]);
    });
  for (auto &x : th) x.join();
  for (int q = 0; q < tot; ++q)
    if (!ok[q]) return fail(RP_EINVAL, "field " + std::to_string(q % nB) + ": " + msgs[q]);
  return RP_OK;
}

// Term kernel for a system: index pairs (complex FP32, at least 8 leading spin-1/2 nuclei),
// the 256-index tile, or the generic mixed-radix form.
template <typename R>
static int term_kind_of(const SysArgs<R> &sa, const Opts &op) {
  int kind = sa.tiled ? kTermTile : kTermGen;
  if (std::is_same<R, float>::value && sa.tiled && sa.nhalf >= 8 && !(op.flags & RP_FLAG_TERM_SCALAR))
    kind = kTermPair;
  return kind;
}

// One system of a tiled propagation: spec in the internal axis order, its fields (host),
// angles (device) and the index of its first output.
struct TiledSys {
  SystemSpec spec;
  const double *B = nullptr;
  const double *angles = nullptr;
  int64_t out = 0;
};

// Tiled propagation of every (system, field, sample) job of a group of systems that share a
// term kernel, as a persistent job queue.  The workspace holds a fixed set of slots, one
// wavepacket each; the slots of one nuclear-state count Z form a pool.  Every Chebyshev term
// is one launch over the tiles of all occupied slots, whatever their Z.  When a job has done
// its steps, its yield is written out and the next job of the pool's queue (longest first)
// takes the slot, starting at its own step 0, so the launches stay full until the queues
// drain.  The host knows every job's step count, so it updates the slot tables between steps
// without waiting for the device.  Pools get slots in proportion to the steps their jobs need,
// so that they drain together.  While the occupied slots are a prefix of one system's pool the
// kernels run in their uniform form (job = tile / nbx, system constants in the kernel
// arguments); otherwise per tile they read the slot index and the slot's descriptor (offsets,
// field, coherent-state row) and the system's constants from a table.
template <typename R>
struct TiledRun {
  struct Job {
    int32_t sys, field, sample;
  };
  struct Pool {
    int64_t Z = 0, nbx = 0, slots = 0, slot0 = 0;
    std::vector<int64_t> queue;   // job indices, decreasing step count
  };
  std::vector<TiledSys> sys;
  int nB = 0;
  int64_t M = 0;
  int nt = 1, rcw = 8, rkp = 8, kind = kTermGen, remap = 0;
  std::vector<FieldDev<R>> fdev;
  std::vector<cx<R>> coef;
  std::vector<R> ell;
  std::vector<double> dts, sys_k;
  std::vector<int64_t> nsteps, tab_off;
  std::vector<SysArgs<R>> sargs;
  int64_t tab_rows = 0;
  std::vector<Job> jobs;
  std::vector<Pool> pools;
  int64_t n_slots = 0, slot_states = 0, slot_tiles = 0;   // slots, sum of their Z and of their tiles
  int64_t fixed_bytes = 0, chunk_bytes = 0;

  static int64_t nbx_of(int64_t Z) { return (Z + kBlock - 1) / kBlock; }
  int64_t slots_size(int64_t ns, int64_t sZ, int64_t tiles) const {
    Sizer z;
    for (int b = 0; b < 3; ++b) z.add<cx<R>>(4 * sZ);       // psi / phi_even, phi_odd, accumulator
    z.add<cx<R>>((int64_t)nt * sZ);                          // singlet amplitudes of one step
    z.add<double>(tiles);                                    // norm partials
    z.add<double>(2 * tiles);                                // quadrature partials
    z.add<int32_t>(tiles);                                   // tile -> slot of the term launches
    z.add<int32_t>(2 * tiles);                               // (slot, tile) of the initialisation launches
    z.add<double>(ns);                                       // phi
    z.add<double>(ns);                                       // previous norm
    z.add<int32_t>(ns);                                      // steps done
    z.add<int32_t>(ns);                                      // field of each slot's job
    z.add<int64_t>(ns);                                      // output index
    z.add<QJob>(ns);
    for (int l = 0; l < 3; ++l) z.add<int32_t>(ns);          // occupied, finished and refilled slots
    return z.used;
  }

  // Slots per pool for a total of E nuclear states (at least one per pool, at most its jobs),
  // in proportion to the steps of each pool's jobs.
  void assign_slots(double E, const std::vector<double> &steps) {
    double denom = 0.0;
    for (size_t p = 0; p < pools.size(); ++p) denom += steps[p] * (double)pools[p].Z;
    for (size_t p = 0; p < pools.size(); ++p) {
      const double want = E * steps[p] / std::max(denom, 1.0);
      pools[p].slots = std::max<int64_t>(1, std::min<int64_t>((int64_t)pools[p].queue.size(), (int64_t)want));
    }
    n_slots = slot_states = slot_tiles = 0;
    for (auto &p : pools) {
      p.slot0 = n_slots;
      n_slots += p.slots;
      slot_states += p.slots * p.Z;
      slot_tiles += p.slots * p.nbx;
    }
  }

  int prepare(const Opts &op, int64_t budget, bool tables_in_budget, bool default_chunks) {
    const int ns = (int)sys.size();
    std::vector<const SystemSpec *> specs;
    std::vector<const double *> Bs;
    for (auto &s : sys) {
      specs.push_back(&s.spec);
      Bs.push_back(s.B);
    }
    std::vector<FieldPlan> plans;
    int rc = plan_many(specs, Bs, nB, op, plans);
    if (rc) return rc;
    int rk = 1;
    for (auto &p : plans) {
      nt = std::max(nt, p.n_terms);
      rk = std::max(rk, p.rank);
    }
    // Pad the term count so that (nt - 2) is a multiple of 3: the accumulator is updated
    // by the first launch (terms 0, 1) and then by every third launch (three terms each).
    while ((nt - 2) % 3 != 0) ++nt;
    // The quadrature makes passes of rcw <= 64 (FP32) or 32 (FP64) columns, each reading every
    // singlet amplitude once: the fewest passes that cover the rank, of equal width (a multiple
    // of 16 in FP32, of 8 in FP64), with the rank padded by zero columns to passes * rcw.
    const int wmax = sizeof(R) == 4 ? 64 : 32;
    const int passes = (rk + wmax - 1) / wmax;
    const int align = sizeof(R) == 4 ? 16 : 8;   // FP32: whole column blocks of the MFMA kernel
    rcw = ((rk + passes - 1) / passes + align - 1) / align * align;
    rkp = passes * rcw;
    const int nG = ns * nB;
    fdev.assign(nG, FieldDev<R>());
    coef.assign((size_t)nG * nt, cx<R>{R(0), R(0)});
    ell.assign((size_t)nG * nt * rkp, R(0));
    dts.assign(nG, 0.0);
    nsteps.assign(nG, 0);
    sargs.resize(ns);
    sys_k.assign(2 * ns, 0.0);
    tab_off.assign(ns, 0);
    int64_t max_vec = 0;
    for (int s = 0; s < ns; ++s) {
      const SystemSpec &sp = sys[s].spec;
      sargs[s] = make_sysargs<R>(sp);
      sys_k[2 * s] = sp.kS;
      sys_k[2 * s + 1] = std::min(sp.kS, sp.kT);
      tab_off[s] = tab_rows;
      tab_rows += M * std::max(sp.N(), 1);
      max_vec = std::max<int64_t>(max_vec, 4 * sp.Z * (int64_t)sizeof(cx<R>));
      const double dk = std::fabs(sp.kS - sp.kT);
      for (int b = 0; b < nB; ++b) {
        const int g = s * nB + b;
        const FieldPlan &p = plans[g];
        FieldDev<R> d;
        d.omega = (R)p.omega;
        d.c_re = (R)p.c_re;
        d.c_im = (R)(p.c_im + (sp.kS >= sp.kT ? 0.0 : 0.5 * dk));
        d.s1 = (R)(1.0 / p.r);
        d.s2 = (R)(2.0 / p.r);
        fdev[g] = d;
        for (int n = 0; n < p.n_terms; ++n) coef[(size_t)g * nt + n] = {(R)p.coef[n].real(), (R)p.coef[n].imag()};
        for (int n = 0; n < p.n_terms; ++n)
          for (int r = 0; r < p.rank; ++r) ell[((size_t)g * nt + n) * rkp + r] = (R)p.ell[(size_t)n * p.rank + r];
        dts[g] = p.dt;
        nsteps[g] = p.n_steps;
      }
    }
    // Jobs, and one queue per nuclear-state count, longest first (stable among equals:
    // system, field, sample order).
    jobs.clear();
    for (int s = 0; s < ns; ++s)
      for (int b = 0; b < nB; ++b)
        for (int64_t m = 0; m < M; ++m) jobs.push_back({s, s * nB + b, (int32_t)m});
    std::vector<int64_t> order(jobs.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t a, int64_t b) { return nsteps[jobs[a].field] > nsteps[jobs[b].field]; });
    pools.clear();
    std::map<int64_t, size_t> pool_of;
    for (int64_t j : order) {
      const int64_t Z = sys[jobs[j].sys].spec.Z;
      auto it = pool_of.find(Z);
      if (it == pool_of.end()) {
        it = pool_of.emplace(Z, pools.size()).first;
        pools.emplace_back();
        pools.back().Z = Z;
        pools.back().nbx = nbx_of(Z);
      }
      pools[it->second].queue.push_back(j);
    }
    std::vector<double> steps(pools.size(), 0.0);
    for (size_t p = 0; p < pools.size(); ++p)
      for (int64_t j : pools[p].queue) steps[p] += (double)nsteps[jobs[j].field];
    Sizer f;
    f.add<FieldDev<R>>(nG);
    f.add<cx<R>>((int64_t)coef.size());
    f.add<R>((int64_t)ell.size());
    f.add<double>(nG);
    f.add<SysArgs<R>>(ns);
    f.add<double>(2 * ns);
    f.add<cx<double>>(tab_rows * (RP_MAX_TWO_I + 1));
    fixed_bytes = f.used;
    const int64_t region = tables_in_budget ? budget - fixed_bytes : budget;
    // Slots: by default the three wavepacket buffers take about 192 MB (resident in the 256 MB
    // Infinity Cache across launches) or 64 wavepackets of the typical size, whichever is
    // more; then as many as the workspace holds, and fewer than 2^24 tiles per launch.
    double typical = 0.0, wsum = 0.0;
    for (size_t p = 0; p < pools.size(); ++p) {
      typical += steps[p] * (double)pools[p].Z;
      wsum += steps[p];
    }
    typical /= std::max(wsum, 1.0);
    double E = std::max((double)(((int64_t)192 << 20) / (12 * (int64_t)sizeof(cx<R>))), 64.0 * typical);
    if (!default_chunks) E = 1e30;
    assign_slots(E, steps);
    while (slots_size(n_slots, slot_states, slot_tiles) > region || slot_tiles >= ((int64_t)1 << 24)) {
      bool all_one = true;
      for (auto &p : pools) all_one = all_one && p.slots == 1;
      if (all_one)
        return fail(RP_ENOMEM, "workspace of " + std::to_string(budget) + " bytes is too small for one wavepacket of " +
                                   "each of " + std::to_string(pools.size()) + " state sizes (needs " +
                                   std::to_string(fixed_bytes + slots_size(n_slots, slot_states, slot_tiles)) + ")");
      E = std::min(E, (double)slot_states) * 0.9;
      assign_slots(E, steps);
    }
    chunk_bytes = slots_size(n_slots, slot_states, slot_tiles);
    // Block order: each XCD takes a contiguous eighth of the launch's tiles (whole wavepackets
    // when there are eight or more, whose partner tiles then stay in one L2) unless a
    // wavepacket exceeds 32 MB; such states are spread round-robin over the XCDs, so that the
    // whole GPU works on few wavepackets at a time and far partners hit the Infinity Cache.
    // (Measured: contiguous ranges gain 3-19 % from 2^16 to 2^20 spin-1/2 states; round-robin
    // gains 5 % on a 95 MB spin-1 state.)
    remap = max_vec <= ((int64_t)32 << 20) ? 1 : 0;
    if (op.flags & RP_FLAG_XCD_LOCAL) remap = 1;
    if (op.flags & RP_FLAG_XCD_SPREAD) remap = 0;
    return RP_OK;
  }

  int run(Arena &ar, const Opts &op, double *phi_out, double *ps_out, int *flag, bool use_graph, hipStream_t st,
          EventLog &log) {
    const int ns = (int)sys.size();
    const int nG = ns * nB;
    FieldDev<R> *dF = ar.take<FieldDev<R>>(nG);
    cx<R> *dCoef = ar.take<cx<R>>((int64_t)coef.size());
    R *dEll = ar.take<R>((int64_t)ell.size());
    double *dDt = ar.take<double>(nG);
    SysArgs<R> *dSys = ar.take<SysArgs<R>>(ns);
    double *dK = ar.take<double>(2 * ns);
    cx<double> *dTab = ar.take<cx<double>>(tab_rows * (RP_MAX_TWO_I + 1));
    cx<R> *bufs[3];
    for (int b = 0; b < 3; ++b) bufs[b] = ar.take<cx<R>>(4 * slot_states);
    cx<R> *D = ar.take<cx<R>>((int64_t)nt * slot_states);
    double *dPn = ar.take<double>(slot_tiles);
    double *dPq = ar.take<double>(2 * slot_tiles);
    int32_t *dTileJob = ar.take<int32_t>(slot_tiles);
    int32_t *dInitMap = ar.take<int32_t>(2 * slot_tiles);
    double *dPhi = ar.take<double>(n_slots);
    double *dPrev = ar.take<double>(n_slots);
    int32_t *dStep = ar.take<int32_t>(n_slots);
    int32_t *dJf = ar.take<int32_t>(n_slots);
    int64_t *dDst = ar.take<int64_t>(n_slots);
    QJob *dJobs = ar.take<QJob>(n_slots);
    int32_t *dActive = ar.take<int32_t>(n_slots);
    int32_t *dDone = ar.take<int32_t>(n_slots);
    int32_t *dNew = ar.take<int32_t>(n_slots);
    if (ar.overflow) return fail(RP_ENOMEM, "internal: workspace layout overflow");
    HIPCHK(hipMemcpyAsync(dF, fdev.data(), nG * sizeof(FieldDev<R>), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(dCoef, coef.data(), coef.size() * sizeof(cx<R>), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(dEll, ell.data(), ell.size() * sizeof(R), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(dDt, dts.data(), nG * 8, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(dSys, sargs.data(), ns * sizeof(SysArgs<R>), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(dK, sys_k.data(), 2 * ns * 8, hipMemcpyHostToDevice, st));
    for (int s = 0; s < ns; ++s) {
      const SystemSpec &sp = sys[s].spec;
      if (ps_out) {   // time points past a field's last step stay NaN
        const int64_t n = (int64_t)nB * M * op.ps_len;
        hipLaunchKernelGGL(k_fill, dim3(grid1(n)), dim3(256), 0, st, ps_out + sys[s].out * op.ps_len, n, std::nan(""));
        HIPCHK(hipGetLastError());
      }
      // Coherent-state components of every sample (shared by all fields).
      const int N = sp.N();
      if (N > 0 && M > 0) {
        CohArgs ca;
        std::memset(&ca, 0, sizeof(ca));
        ca.angles = sys[s].angles;
        ca.tab = dTab + tab_off[s] * (RP_MAX_TWO_I + 1);
        ca.M = M;
        ca.N = N;
        ca.mode = op.init_mode;
        for (int k = 0; k < N; ++k) {
          ca.two_I[k] = sp.two_I[k];
          ca.perm[k] = sp.perm[k];
        }
        hipLaunchKernelGGL(k_coherent, dim3(grid1(M * N)), dim3(256), 0, st, ca);
        HIPCHK(hipGetLastError());
      }
    }
    // Static slot layout: pool by pool, slot s of a pool at vec/amp offsets of its own.
    std::vector<int32_t> slot_pool(n_slots);
    std::vector<int64_t> slot_vec(n_slots), slot_amp(n_slots);
    {
      int64_t vec = 0, amp = 0;
      for (size_t p = 0; p < pools.size(); ++p)
        for (int64_t q = 0; q < pools[p].slots; ++q) {
          const int64_t s = pools[p].slot0 + q;
          slot_pool[s] = (int32_t)p;
          slot_vec[s] = vec;
          slot_amp[s] = amp;
          vec += 4 * pools[p].Z;
          amp += pools[p].Z;
        }
    }
    const bool one_system = ns == 1;
    const int64_t Z0 = sys[0].spec.Z, nbx0 = nbx_of(Z0);
    const SysArgs<R> &sa0 = sargs[0];
    std::vector<int64_t> slot_job(n_slots, -1), slot_left(n_slots, 0);
    std::vector<size_t> next(pools.size(), 0);
    std::vector<int32_t> hJf(n_slots, 0), hTile, hInit, active, done, fresh;
    std::vector<int64_t> hDst(n_slots, 0);
    std::vector<QJob> hJobs(n_slots);
    std::memset(hJobs.data(), 0, n_slots * sizeof(QJob));
    for (int64_t s = 0; s < n_slots; ++s) {
      const Pool &p = pools[slot_pool[s]];
      hJobs[s].nbx = (int32_t)p.nbx;
      hJobs[s].Z = p.Z;
      hJobs[s].vec = slot_vec[s];
      hJobs[s].amp = slot_amp[s];
    }
    // Takes the next job of slot s's pool, if any.
    auto assign = [&](int64_t s) -> bool {
      Pool &p = pools[slot_pool[s]];
      size_t &k = next[slot_pool[s]];
      if (k >= p.queue.size()) {
        slot_job[s] = -1;
        return false;
      }
      const int64_t j = p.queue[k++];
      const Job &jb = jobs[j];
      slot_job[s] = j;
      slot_left[s] = nsteps[jb.field];
      hJf[s] = jb.field;
      hDst[s] = sys[jb.sys].out + (int64_t)(jb.field - jb.sys * nB) * M + jb.sample;
      hJobs[s].sys = jb.sys;
      hJobs[s].field = jb.field;
      hJobs[s].tab = tab_off[jb.sys] + (int64_t)jb.sample * std::max(sys[jb.sys].spec.N(), 1);
      return true;
    };
    // Starts the jobs just assigned to the slots in `fresh`: tables, cleared sums, psi_0 into
    // buffer ipsi.
    auto start = [&](int ipsi) -> int {
      if (fresh.empty()) return RP_OK;
      HIPCHK(hipMemcpyAsync(dJf, hJf.data(), n_slots * 4, hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(dDst, hDst.data(), n_slots * 8, hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(dJobs, hJobs.data(), n_slots * sizeof(QJob), hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(dNew, fresh.data(), fresh.size() * 4, hipMemcpyHostToDevice, st));
      hInit.clear();
      for (int32_t s : fresh)
        for (int64_t b = 0; b < hJobs[s].nbx; ++b) {
          hInit.push_back(s);
          hInit.push_back((int32_t)b);
        }
      HIPCHK(hipMemcpyAsync(dInitMap, hInit.data(), hInit.size() * 4, hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(k_slots_reset, dim3(grid1((int64_t)fresh.size())), dim3(256), 0, st, (const int32_t *)dNew,
                         (int64_t)fresh.size(), dPhi, dPrev, dStep);
      InitArgs<R> ia;
      std::memset(&ia, 0, sizeof(ia));
      ia.psi = bufs[ipsi];
      ia.tab = dTab;
      ia.init_map = dInitMap;
      ia.jobs = dJobs;
      ia.systab = dSys;
      ia.tiles = (int64_t)hInit.size() / 2;
      hipLaunchKernelGGL((k_init<R, true>), dim3((unsigned)ia.tiles), dim3(kBlock), 0, st, ia);
      HIPCHK(hipGetLastError());
      fresh.clear();
      return RP_OK;
    };
    // Occupied slots in slot order; their tiles numbered in that order for the term launches.
    auto relayout = [&]() -> int {
      active.clear();
      hTile.clear();
      for (int64_t s = 0; s < n_slots; ++s)
        if (slot_job[s] >= 0) {
          hJobs[s].blk = (int64_t)hTile.size();
          for (int64_t b = 0; b < hJobs[s].nbx; ++b) hTile.push_back((int32_t)s);
          active.push_back((int32_t)s);
        }
      if (active.empty()) return RP_OK;
      HIPCHK(hipMemcpyAsync(dJobs, hJobs.data(), n_slots * sizeof(QJob), hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(dTileJob, hTile.data(), hTile.size() * 4, hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(dActive, active.data(), active.size() * 4, hipMemcpyHostToDevice, st));
      return RP_OK;
    };
    int rc;
    int ip = 0, ia_ = 2, iodd = 1;   // psi, accumulator and odd-term buffers
    for (int64_t s = 0; s < n_slots; ++s)
      if (assign(s)) fresh.push_back((int32_t)s);
    if ((rc = start(ip))) return rc;
    if ((rc = relayout())) return rc;
    const double rtol = op.precision == 64 ? 1e-9 : 1e-4;
    const double eb = (double)sizeof(R) / 4.0;   // bytes per element, in units of complex-FP32 bytes
    const int64_t slab = slot_states;
    // Streaming (non-temporal) loads and stores of phi_{n-1}, phi_{n+1} and the accumulator
    // when the slots' three wavepacket buffers exceed the 256 MB Infinity Cache: they would not
    // survive there until the next launch anyway, and the hint leaves the L2 to the partner
    // tiles of phi_n.  The singlet amplitudes, read only by the quadrature, always stream.
    const bool stream_nt = 3 * 4 * slot_states * (int64_t)sizeof(cx<R>) > ((int64_t)256 << 20);
    // All launches of one step over the occupied slots: Chebyshev terms, in-step quadrature,
    // finalisation.  uniform: the occupied slots are slots 0 .. n-1 of the only system.
    auto enqueue_step = [&](int64_t tiles, int64_t n_act, bool uniform, int ipsi, int iacc) {
      const bool q = !uniform;
      const unsigned grid = (unsigned)tiles;
      TermArgs<R> ta;
      std::memset(&ta, 0, sizeof(ta));
      ta.fields = dF;
      ta.coef = dCoef;
      ta.job_field = dJf;
      ta.part_norm = dPn;
      ta.tile_job = dTileJob;
      ta.jobs = dJobs;
      ta.systab = dSys;
      ta.nbx = nbx0;
      ta.tiles = tiles;
      ta.njobs = (int32_t)n_act;
      ta.n_terms = nt;
      ta.remap = remap;
      ta.acc = bufs[iacc];
      cx<R> *even = bufs[ipsi], *odd = bufs[iodd];
      // n = 0: phi_1 = Gh phi_0
      ta.phin = even;
      ta.phio = odd;
      ta.n = 0;
      ta.dnext = D + slab;
      ta.dfirst = D;
      log.mark(st);
      launch_term<R>(kFirst, kind, stream_nt, q, grid, st, ta, sa0);
      double bytes = 28.0 * eb;
      for (int n = 1; n + 1 < nt; ++n) {
        // phi_{n+1} = 2 Gh phi_n - phi_{n-1}, written over phi_{n-1}; every third launch also
        // adds phi_{n-1}, phi_n, phi_{n+1} to the step accumulator.
        ta.phin = (n & 1) ? odd : even;
        ta.phio = (n & 1) ? even : odd;
        ta.n = n;
        ta.dnext = D + (int64_t)(n + 1) * slab;
        const bool acc3 = (n % 3) == 0;
        launch_term<R>(acc3 ? kAcc3 : kPlain, kind, stream_nt, q, grid, st, ta, sa0);
        bytes += (acc3 ? 42.0 : 26.0) * eb;
      }
      log.mark(st);
      log.close(0);
      if (log.on) {
        double el = 0.0;   // wavepacket elements of the launch
        for (int32_t s : active) el += 4.0 * (double)hJobs[s].Z;
        g_prof.term_launches += nt - 1;
        g_prof.elems += (double)(nt - 1) * el;
        g_prof.bytes += bytes * el;
        g_prof.quad_launches += 1;
        g_prof.terms = nt;
      }
      QuadArgs<R> qa;
      std::memset(&qa, 0, sizeof(qa));
      qa.d = D;
      qa.slab = slab;
      qa.ell = dEll;
      qa.job_field = dJf;
      qa.part = dPq;
      qa.tile_job = dTileJob;
      qa.jobs = dJobs;
      qa.Z = Z0;
      qa.nbx = nbx0;
      qa.tiles = tiles;
      qa.njobs = (int32_t)n_act;
      qa.n_terms = nt;
      qa.rank_pad = rkp;
      qa.remap = remap;
      log.mark(st);
      launch_quad<R>(rcw, q, grid, st, qa);
      log.mark(st);
      log.close(1);
      FinArgs fa;
      std::memset(&fa, 0, sizeof(fa));
      fa.part_q = dPq;
      fa.part_norm = dPn;
      fa.phi = dPhi;
      fa.prev_norm = dPrev;
      fa.flag = flag;
      fa.job_field = dJf;
      fa.dt = dDt;
      fa.stepc = dStep;
      fa.jobs = q ? dJobs : nullptr;
      fa.slots = q ? dActive : nullptr;
      fa.sys_k = dK;
      fa.nbx = nbx0;
      fa.njobs = (int32_t)n_act;
      fa.kS = sys[0].spec.kS;
      fa.kmin = std::min(sys[0].spec.kS, sys[0].spec.kT);
      fa.rtol = rtol;
      fa.ps_t = ps_out;
      fa.dst = dDst;
      fa.ps_len = op.ps_len;
      hipLaunchKernelGGL(k_finalize, dim3((unsigned)n_act), dim3(kBlock), 0, st, fa);
    };
    // One captured graph per (tiles, occupied slots, form, buffer parity), replayed while the
    // occupied set keeps its shape; the slot tables it reads are updated between steps.
    using GraphKey = std::tuple<int64_t, int64_t, int, int>;
    std::map<GraphKey, hipGraphExec_t> graphs;
    // HIP does not promise that destroying an executable graph waits for its launches, so the
    // call's launches are waited for before its graphs are destroyed.
    struct GraphsGuard {
      std::map<GraphKey, hipGraphExec_t> &g;
      hipStream_t s;
      ~GraphsGuard() {
        if (g.empty()) return;
        (void)hipStreamSynchronize(s);
        for (auto &kv : g) (void)hipGraphExecDestroy(kv.second);
      }
    } graphs_guard{graphs, st};
    while (!active.empty()) {
      const int64_t tiles = (int64_t)hTile.size(), n_act = (int64_t)active.size();
      const bool uniform = one_system && active.back() == n_act - 1;
      if (use_graph) {
        const GraphKey key{tiles, n_act, uniform ? 1 : 0, ip};
        auto it = graphs.find(key);
        if (it == graphs.end()) {
          HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
          enqueue_step(tiles, n_act, uniform, ip, ia_);
          hipGraph_t g = nullptr;
          const hipError_t ec = hipStreamEndCapture(st, &g);
          if (ec != hipSuccess || !g) return fail(RP_EDEVICE, std::string("graph capture: ") + hipGetErrorString(ec));
          hipGraphExec_t ge = nullptr;
          const hipError_t ei = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
          (void)hipGraphDestroy(g);
          if (ei != hipSuccess) return fail(RP_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(ei));
          it = graphs.emplace(key, ge).first;
        }
        HIPCHK(hipGraphLaunch(it->second, st));
      } else {
        enqueue_step(tiles, n_act, uniform, ip, ia_);
        HIPCHK(hipGetLastError());
      }
      std::swap(ip, ia_);
      // Jobs that have done their steps: yields out, next jobs in.
      done.clear();
      for (int32_t s : active)
        if (--slot_left[s] == 0) done.push_back(s);
      if (done.empty()) continue;
      HIPCHK(hipMemcpyAsync(dDone, done.data(), done.size() * 4, hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(k_slots_scatter, dim3(grid1((int64_t)done.size())), dim3(256), 0, st, (const int32_t *)dDone,
                         (int64_t)done.size(), (const double *)dPhi, (const int64_t *)dDst, phi_out);
      HIPCHK(hipGetLastError());
      bool emptied = false;
      for (int32_t s : done) {
        if (assign(s)) fresh.push_back(s);
        else emptied = true;
      }
      if ((rc = start(ip))) return rc;
      if (emptied && (rc = relayout())) return rc;
    }
    return RP_OK;
  }
};

// Quadrature columns the resident kernel keeps per thread: 32 up to 512-thread workgroups, 24 for
// 1024 threads (register budget 128 per lane).
static int res_rank_limit(int64_t Z) { return Z > 512 ? 24 : kResRank; }

// Every job of the LDS-resident systems of a call (one launch per workgroup-size class).
template <typename R>
struct ResidentRun {
  std::vector<SystemSpec> specs;
  std::vector<const double *> B, angles;
  std::vector<int64_t> out;          // index of each system's first output
  int nB = 0;
  int64_t M = 0;
  std::vector<ResSys<R>> rsys;
  std::vector<ResField<R>> rf;
  std::vector<cx<R>> coef;
  std::vector<R> ell;
  std::vector<ResJob> all;
  std::vector<int64_t> start;
  int64_t tab_elems = 0;
  int64_t bytes = 0;

  int prepare(const Opts &op) {
    const int ns = (int)specs.size();
    // Plan every (system, field) with a step short enough that the quadrature rank fits kResRank.
    std::vector<FieldPlan> plans((size_t)ns * nB);
    std::vector<std::string> msgs((size_t)ns * nB);
    std::vector<char> ok((size_t)ns * nB, 0);
    {
      const int tot = ns * nB;
      const int nth = std::max(1, std::min<int>(tot, (int)std::thread::hardware_concurrency()));
      std::vector<std::thread> th;
      for (int t = 0; t < nth; ++t)
        th.emplace_back([&, t]() {
          for (int q = t; q < tot; q += nth) {
            const int i = q / nB, b = q % nB;
            const int rmax = res_rank_limit(specs[i].Z);
            double rdt = std::min(op.rdt, 40.0);
            for (int tries = 0; tries < 12; ++tries) {
              ok[q] = plan_field(specs[i], B[i][b], op.tol, rdt, op.r_scale, op.chol_tol, op.max_growth, plans[q],
                                 msgs[q]);
              if (!ok[q] || plans[q].rank <= rmax) break;
              rdt *= 0.75;
            }
            if (ok[q] && plans[q].rank > rmax) {
              ok[q] = 0;
              msgs[q] = "quadrature rank does not fit the resident kernel";
            }
          }
        });
      for (auto &x : th) x.join();
    }
    for (size_t q = 0; q < plans.size(); ++q)
      if (!ok[q]) return fail(RP_EINVAL, "field plan: " + msgs[q]);
    rsys.assign(ns, ResSys<R>());
    rf.assign((size_t)ns * nB, ResField<R>());
    coef.clear();
    ell.clear();
    tab_elems = 0;
    const double rtol = op.precision == 64 ? 1e-9 : 1e-4;
    for (int i = 0; i < ns; ++i) {
      std::memset(&rsys[i], 0, sizeof(ResSys<R>));
      rsys[i].sa = make_sysargs<R>(specs[i]);
      rsys[i].tab_off = tab_elems;
      rsys[i].kS = specs[i].kS;
      rsys[i].kmin = std::min(specs[i].kS, specs[i].kT);
      rsys[i].rtol = rtol;
      tab_elems += M * std::max(specs[i].N(), 1) * (RP_MAX_TWO_I + 1);
      const double dk = std::fabs(specs[i].kS - specs[i].kT);
      for (int b = 0; b < nB; ++b) {
        const FieldPlan &p = plans[(size_t)i * nB + b];
        ResField<R> &f = rf[(size_t)i * nB + b];
        std::memset(&f, 0, sizeof(f));
        f.fd.omega = (R)p.omega;
        f.fd.c_re = (R)p.c_re;
        f.fd.c_im = (R)(p.c_im + (specs[i].kS >= specs[i].kT ? 0.0 : 0.5 * dk));
        f.fd.s1 = (R)(1.0 / p.r);
        f.fd.s2 = (R)(2.0 / p.r);
        f.dt = p.dt;
        f.n_steps = (int32_t)p.n_steps;
        f.n_terms = p.n_terms;
        f.coef_off = (int64_t)coef.size();
        for (int n = 0; n < p.n_terms; ++n) coef.push_back({(R)p.coef[n].real(), (R)p.coef[n].imag()});
        f.ell_off = (int64_t)ell.size();
        for (int n = 0; n < p.n_terms; ++n)
          for (int r = 0; r < kResRank; ++r) ell.push_back(r < p.rank ? (R)p.ell[(size_t)n * p.rank + r] : R(0));
      }
    }
    // Jobs grouped by workgroup size (next power of two >= max(64, Z)), longest first.
    std::vector<std::vector<ResJob>> groups(5);   // 64, 128, 256, 512, 1024
    std::vector<std::vector<double>> costs(5);
    for (int i = 0; i < ns; ++i) {
      int g = 0;
      while ((64 << g) < specs[i].Z) ++g;
      for (int b = 0; b < nB; ++b) {
        const FieldPlan &p = plans[(size_t)i * nB + b];
        for (int64_t s = 0; s < M; ++s) {
          ResJob j;
          j.sys = i;
          j.field = i * nB + b;
          j.sample = (int32_t)s;
          j.pad = 0;
          j.out = out[i] + (int64_t)b * M + s;
          groups[g].push_back(j);
          costs[g].push_back((double)p.n_steps * p.n_terms);
        }
      }
    }
    all.clear();
    start.assign(6, 0);
    for (int g = 0; g < 5; ++g) {
      std::vector<size_t> ord(groups[g].size());
      std::iota(ord.begin(), ord.end(), 0);
      std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return costs[g][a] > costs[g][b]; });
      for (size_t q : ord) all.push_back(groups[g][q]);
      start[g + 1] = (int64_t)all.size();
    }
    Sizer z;
    z.add<ResSys<R>>(ns);
    z.add<ResField<R>>((int64_t)rf.size());
    z.add<cx<R>>((int64_t)coef.size());
    z.add<R>((int64_t)ell.size());
    z.add<cx<double>>(tab_elems);
    z.add<ResJob>((int64_t)all.size());
    bytes = z.used;
    return RP_OK;
  }

  int run(Arena &ar, const Opts &op, double *phi, int *flag, hipStream_t st) {
    const int ns = (int)specs.size();
    ResSys<R> *dS = ar.take<ResSys<R>>(ns);
    ResField<R> *dF = ar.take<ResField<R>>((int64_t)rf.size());
    cx<R> *dC = ar.take<cx<R>>((int64_t)coef.size());
    R *dE = ar.take<R>((int64_t)ell.size());
    cx<double> *dT = ar.take<cx<double>>(tab_elems);
    ResJob *dJ = ar.take<ResJob>((int64_t)all.size());
    if (ar.overflow) return fail(RP_ENOMEM, "internal: workspace layout overflow");
    HIPCHK(hipMemcpyAsync(dS, rsys.data(), rsys.size() * sizeof(ResSys<R>), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(dF, rf.data(), rf.size() * sizeof(ResField<R>), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(dC, coef.data(), coef.size() * sizeof(cx<R>), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(dE, ell.data(), ell.size() * sizeof(R), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(dJ, all.data(), all.size() * sizeof(ResJob), hipMemcpyHostToDevice, st));
    for (int i = 0; i < ns; ++i) {
      const int N = specs[i].N();
      CohArgs ca;
      std::memset(&ca, 0, sizeof(ca));
      ca.angles = angles[i];
      ca.tab = dT + rsys[i].tab_off;
      ca.M = M;
      ca.N = N;
      ca.mode = op.init_mode;
      for (int k = 0; k < N; ++k) {
        ca.two_I[k] = specs[i].two_I[k];
        ca.perm[k] = specs[i].perm[k];
      }
      if (N > 0) hipLaunchKernelGGL(k_coherent, dim3(grid1(M * N)), dim3(256), 0, st, ca);
    }
    HIPCHK(hipGetLastError());
    for (int g = 0; g < 5; ++g) {
      const int64_t n = start[g + 1] - start[g];
      if (n == 0) continue;
      const int Zb = 64 << g;
      ResArgs<R> ra;
      ra.sys = dS;
      ra.fields = dF;
      ra.jobs = dJ + start[g];
      ra.coef = dC;
      ra.ell = dE;
      ra.tab = dT;
      ra.phi = phi;
      ra.flag = flag;
      ra.njobs = n;
      const size_t shmem = 2 * 4 * (size_t)Zb * sizeof(cx<R>);
      if (Zb > 512) {
        HIPCHK(hipFuncSetAttribute((const void *)k_resident<R, 1024, 24>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)shmem));
        hipLaunchKernelGGL((k_resident<R, 1024, 24>), dim3((unsigned)n), dim3(Zb), shmem, st, ra);
      } else {
        HIPCHK(hipFuncSetAttribute((const void *)k_resident<R, 512, kResRank>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
        hipLaunchKernelGGL((k_resident<R, 512, kResRank>), dim3((unsigned)n), dim3(Zb), shmem, st, ra);
      }
      HIPCHK(hipGetLastError());
    }
    return RP_OK;
  }
};

// The Chebyshev path of rp_propagate (and of its variant on the static scratch area): plans
// every system, sizes one workspace for the call, then runs the LDS-resident systems and the
// tiled groups one after another on the caller's stream (each part reuses the same workspace:
// stream order separates them).  scratch: device memory of scratch_bytes to use instead of an
// allocation (nullptr: one stream-ordered allocation for the call).
template <typename R>
static int propagate_chebyshev(const rp_system *sys, int n_sys, const double *B_mT, int nB, const double *angles,
                               int64_t M, const Opts &op, double *phi, double *ps_t, hipStream_t st, EventLog &log,
                               char *scratch, int64_t scratch_bytes) {
  std::vector<int64_t> aoffs(n_sys, 0);
  {
    int64_t o = 0;
    for (int i = 0; i < n_sys; ++i) {
      aoffs[i] = o;
      o += M * (sys[i].n_nuc[0] + sys[i].n_nuc[1]) * 2;
    }
  }
  // Systems small enough for the LDS-resident kernel run together in one launch per size class;
  // the rest run tiled, grouped by term kernel (one job queue per group).
  const int64_t zmax = sizeof(R) == 8 ? kResMax64 : kResMax32;
  ResidentRun<R> res;
  res.nB = nB;
  res.M = M;
  std::vector<TiledRun<R>> groups;
  std::vector<int> group_kind;
  for (int i = 0; i < n_sys; ++i) {
    const rp_system *s = &sys[i];
    SystemSpec spec = tile_order(make_spec(s->n_nuc[0], s->n_nuc[1], s->two_I, s->a_mT, s->J_mT, s->kS, s->kT,
                                           s->T_us, gamma_of(s)),
                                 (op.flags & RP_FLAG_AXES_HIGH_FIRST) != 0);
    const double *ang = angles ? angles + aoffs[i] : nullptr;
    if (!(op.flags & RP_FLAG_TILED) && !log.on && !ps_t && spec.Z <= zmax) {
      res.specs.push_back(spec);
      res.B.push_back(B_mT + (int64_t)i * nB);
      res.angles.push_back(ang);
      res.out.push_back((int64_t)i * nB * M);
      continue;
    }
    const int kind = term_kind_of(make_sysargs<R>(spec), op);
    size_t g = 0;
    while (g < groups.size() && group_kind[g] != kind) ++g;
    if (g == groups.size()) {
      groups.emplace_back();
      groups.back().nB = nB;
      groups.back().M = M;
      groups.back().kind = kind;
      group_kind.push_back(kind);
    }
    TiledSys ts;
    ts.spec = spec;
    ts.B = B_mT + (int64_t)i * nB;
    ts.angles = ang;
    ts.out = (int64_t)i * nB * M;
    groups[g].sys.push_back(ts);
  }
  int rc;
  int64_t need = 0;
  if (!res.specs.empty()) {
    if ((rc = res.prepare(op))) return rc;
    need = res.bytes;
  }
  // Workspace budget: the caller's cap, else half of the free device memory; the static
  // scratch area when there is one.
  int64_t budget = scratch ? scratch_bytes : op.workspace;
  if (budget <= 0) {
    size_t fr = 0, tot = 0;
    HIPCHK(hipMemGetInfo(&fr, &tot));
    budget = (int64_t)(fr / 2);
  }
  const int64_t flag_bytes = 256;
  if (scratch && need + flag_bytes > budget)   // (an allocated workspace takes the small resident tables beyond the cap)
    return fail(RP_ENOMEM, "workspace of " + std::to_string(budget) + " bytes is too small for the LDS-resident jobs (" +
                               std::to_string(need + flag_bytes) + " needed)");
  for (auto &g : groups) {
    // An explicit cap (opts->workspace_bytes) bounds the chunk buffers; the call's tables come
    // on top.  The static area and the default budget hold everything.
    const bool capped = !scratch && op.workspace > 0;
    if ((rc = g.prepare(op, capped ? budget : budget - flag_bytes, !capped, op.workspace <= 0))) return rc;
    need = std::max(need, g.fixed_bytes + g.chunk_bytes);
  }
  need += flag_bytes;
  // One block for the call: stream-ordered, freed on the stream when the call ends.
  struct Block {
    void *p = nullptr;
    hipStream_t s = nullptr;
    bool async = false;
    ~Block() {
      if (!p) return;
      if (async) (void)hipFreeAsync(p, s);
      else (void)hipFree(p);
    }
  } blk;
  char *base = scratch;
  if (!scratch) {
    blk.s = st;
    if (hipMallocAsync(&blk.p, (size_t)need, st) == hipSuccess) {
      blk.async = true;
    } else {
      (void)hipGetLastError();
      if (hipMalloc(&blk.p, (size_t)need) != hipSuccess) {
        (void)hipGetLastError();
        blk.p = nullptr;
        return fail(RP_ENOMEM, "device workspace of " + std::to_string(need) + " bytes could not be allocated");
      }
    }
    base = (char *)blk.p;
  }
  int *flag = (int *)base;
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(256), 0, st, (int32_t *)flag, 4, 0);
  HIPCHK(hipGetLastError());
  const bool use_graph = !log.on && !(op.flags & RP_FLAG_NO_GRAPH) && !scratch;
  if (!res.specs.empty()) {
    Arena ar{base + flag_bytes, need - flag_bytes, 0, false};
    if ((rc = res.run(ar, op, phi, flag, st))) return rc;
  }
  for (auto &g : groups) {
    Arena ar{base + flag_bytes, need - flag_bytes, 0, false};
    if ((rc = g.run(ar, op, phi, ps_t, flag, use_graph, st, log))) return rc;
  }
  int h_flag = 0;
  HIPCHK(hipMemcpyAsync(&h_flag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (h_flag) return fail(RP_ENOTCONV, "wavepacket norm grew or became NaN (spectral bound violated)");
  return RP_OK;
}

}  // namespace rp

// ============================================================================= C ABI
using namespace rp;

extern "C" const char *rp_strerror(int code) {
  switch (code) {
    case RP_OK: return "ok";
    case RP_EINVAL: return "invalid argument";
    case RP_ENOMEM: return "out of device memory";
    case RP_EDEVICE: return "HIP error";
    case RP_ENOTCONV: return "propagation did not converge (norm grew)";
    case RP_ENOTIMPL: return "not implemented";
    default: return "unknown error";
  }
}

extern "C" const char *rp_last_error(void) { return g_err.c_str(); }

extern "C" int rp_bessel_j(double x, int32_t nmax, double *out) {
  if (!out || nmax < 0 || !(x >= 0.0) || !std::isfinite(x)) return fail(RP_EINVAL, "bad bessel arguments");
  bessel_j(x, nmax, out);
  return RP_OK;
}

extern "C" int rp_plan_field(const rp_system *s, double B_mT, const rp_opts *opts, double *info, double *coef,
                             double *ell) {
  int rc = validate_system(s);
  if (rc) return rc;
  if (!info) return fail(RP_EINVAL, "null info");
  Opts op;
  rc = read_opts(opts, op);
  if (rc) return rc;
  const double g = gamma_of(s);
  SystemSpec spec = make_spec(s->n_nuc[0], s->n_nuc[1], s->two_I, s->a_mT, s->J_mT, s->kS, s->kT, s->T_us, g);
  FieldPlan p;
  std::string msg;
  if (!plan_field(spec, B_mT, op.tol, op.rdt, op.r_scale, op.chol_tol, op.max_growth, p, msg)) return fail(RP_EINVAL, msg);
  info[0] = p.r;
  info[1] = p.c_re;
  info[2] = p.c_im;
  info[3] = p.dt;
  info[4] = (double)p.n_steps;
  info[5] = (double)p.n_terms;
  info[6] = (double)p.rank;
  info[7] = p.x;
  if (coef)
    for (int n = 0; n < p.n_terms; ++n) {
      coef[2 * n] = p.coef[n].real();
      coef[2 * n + 1] = p.coef[n].imag();
    }
  if (ell) std::memcpy(ell, p.ell.data(), p.ell.size() * sizeof(double));
  return RP_OK;
}

extern "C" int64_t rp_design_size(int32_t n_nuclei, int32_t basis_mode) {
  if (n_nuclei < 0 || n_nuclei > RP_MAX_NUCLEI || basis_mode < 0 || basis_mode > 5)
    return fail(RP_EINVAL, "rp_design_size: n_nuclei or basis_mode out of range");
  if (basis_mode < 3) return 1;
  if (basis_mode == 3) return 2;
  int64_t n = 1;
  if (basis_mode == 5) {
    while (n <= n_nuclei) n *= 2;
    return n;
  }
  while (n < n_nuclei) n *= 2;
  return 2 * n;
}

extern "C" int rp_sample(const rp_system *s, uint64_t seed, uint32_t stream_id, uint64_t first_sample, int64_t M,
                         int32_t basis_mode, double *angles, void *hip_stream) {
  int rc = validate_system(s);
  if (rc) return rc;
  if (M < 0) return fail(RP_EINVAL, "M < 0");
  if (basis_mode < 0 || basis_mode > 5) return fail(RP_EINVAL, "basis_mode must be 0 .. 5");
  const int N = s->n_nuc[0] + s->n_nuc[1];
  if (M == 0 || N == 0) return RP_OK;
  if (!angles) return fail(RP_EINVAL, "null angles");
  if (M > ((int64_t)1 << 40) || M * N > ((int64_t)1 << 38)) return fail(RP_EINVAL, "M too large");
  SampleArgs a;
  std::memset(&a, 0, sizeof(a));
  a.angles = angles;
  a.seed = seed;
  a.first = first_sample;
  a.M = M;
  a.N = N;
  a.mode = basis_mode;
  a.stream = stream_id;
  int64_t rad = 1;
  for (int k = 0; k < N; ++k) {
    a.d[k] = s->two_I[k] + 1;
    a.radix[k] = rad;
    rad *= a.d[k];
  }
  a.rows = basis_mode >= 3 ? (uint64_t)rp_design_size(N, basis_mode) : 1;
  hipLaunchKernelGGL(k_sample, dim3(grid1(M * N)), dim3(256), 0, (hipStream_t)hip_stream, a);
  HIPCHK(hipGetLastError());
  return RP_OK;
}

// ----------------------------------------------------------------------------- short-iterative Arnoldi
// The paper's propagator (Sec. III): each step builds an m-dimensional Krylov space of the
// wavepacket under A = H + i beta P_S (the generator without its scalar decay k_T/2, Eq. 1-4),
// projects, and advances by exp(-i H_m dt) with dt chosen from the Arnoldi error estimate.
// It is kept as an alternative to the Chebyshev series for comparison.  Krylov vectors of a
// chunk: [jobs][m + 1][4Z]; every job of a chunk does the same launches, each with its own dt.
constexpr int kSiaMax = 32;   // largest Krylov dimension

// Y = A X for every job (generic mixed-radix form, partners from global memory).
template <typename R>
__global__ __launch_bounds__(256) void k_sia_apply(SysArgs<R> sa, const cx<R> *X, cx<R> *Y, int64_t vstride,
                                                   int64_t nbx, int32_t njobs, const double *omega) {
  const int64_t total = (int64_t)njobs * nbx;
  const int64_t L = xcd_remap(blockIdx.x, total);
  const int64_t job = L / nbx, bx = L - job * nbx;
  const int64_t M = bx * kBlock + threadIdx.x;
  if (M >= sa.Z) return;
  const int64_t Z = sa.Z;
  const cx<R> *x = X + job * vstride;
  const cx<R> zero = {R(0), R(0)};
  const cx<R> x0 = x[M], x1 = x[Z + M], x2 = x[2 * Z + M], x3 = x[3 * Z + M];
  cx<R> y0 = zero, y1 = zero, y2 = zero, y3 = zero;
  R h1 = R(0), h2 = R(0);
  int64_t rem = M;
  for (int k = 0; k < sa.N; ++k) {
    const int64_t st = sa.stride[k];
    const int dk = sa.d[k];
    const int64_t q = rem / dk;
    const int n = (int)(rem - q * dk);
    rem = q;
    const R mk = R(0.5) * R(dk - 1) - R(n);
    const bool r1 = sa.rad[k] == 0;
    if (r1) h1 += sa.a[k] * mk; else h2 += sa.a[k] * mk;
    if (n > 0) {        // partner digit n-1: beta component -> alpha component
      const R fk = sa.f[k][n - 1];
      const cx<R> *p = x + (M - st);
      if (r1) {
        y0 = cadd(y0, cscale(fk, p[2 * Z]));
        y1 = cadd(y1, cscale(fk, p[3 * Z]));
      } else {
        y0 = cadd(y0, cscale(fk, p[Z]));
        y2 = cadd(y2, cscale(fk, p[3 * Z]));
      }
    }
    if (n < dk - 1) {   // partner digit n+1: alpha component -> beta component
      const R fk = sa.f[k][n];
      const cx<R> *p = x + (M + st);
      if (r1) {
        y2 = cadd(y2, cscale(fk, p[0]));
        y3 = cadd(y3, cscale(fk, p[Z]));
      } else {
        y1 = cadd(y1, cscale(fk, p[0]));
        y3 = cadd(y3, cscale(fk, p[2 * Z]));
      }
    }
  }
  const R om = (R)omega[job];
  const R hs = R(0.5) * (h1 + h2), hd = R(0.5) * (h1 - h2), hj = R(0.5) * sa.J;
  y0 = cadd(y0, cscale(om + hs + hj, x0));
  y1 = cadd(y1, cadd(cscale(hd - hj, x1), cscale(sa.J, x2)));
  y2 = cadd(y2, cadd(cscale(-hd - hj, x2), cscale(sa.J, x1)));
  y3 = cadd(y3, cscale(-om - hs + hj, x3));
  const cx<R> t = {R(0.5) * (x1.x - x2.x), R(0.5) * (x1.y - x2.y)};
  const cx<R> ibt = {-sa.beta * t.y, sa.beta * t.x};
  y1 = cadd(y1, ibt);
  y2 = csub(y2, ibt);
  cx<R> *y = Y + job * vstride;
  y[M] = y0;
  y[Z + M] = y1;
  y[2 * Z + M] = y2;
  y[3 * Z + M] = y3;
}

// part[job][bx][i] = sum over the workgroup's indices and the four planes of conj(V_{i0+i}) V_w,
// for i < nd; FP64 accumulation.
template <typename R>
__global__ __launch_bounds__(256) void k_sia_dot(const cx<R> *V, int64_t vstride, int64_t Z, int64_t nbx,
                                                 int32_t njobs, int32_t w, int32_t i0, int32_t nd,
                                                 cx<double> *part) {
  __shared__ double lds[4];
  const int64_t job = blockIdx.x / nbx, bx = blockIdx.x - job * nbx;
  const int64_t M = bx * kBlock + threadIdx.x;
  const bool live = M < Z;
  const cx<R> *v = V + job * vstride;
  cx<R> wv[4];
  for (int e = 0; e < 4; ++e) wv[e] = live ? v[(int64_t)w * 4 * Z + e * Z + M] : cx<R>{R(0), R(0)};
  for (int i = 0; i < nd; ++i) {
    double re = 0.0, im = 0.0;
    if (live)
      for (int e = 0; e < 4; ++e) {
        const cx<R> a = v[(int64_t)(i0 + i) * 4 * Z + e * Z + M];
        re += (double)a.x * wv[e].x + (double)a.y * wv[e].y;
        im += (double)a.x * wv[e].y - (double)a.y * wv[e].x;
      }
    re = block_sum(re, lds);
    im = block_sum(im, lds);
    if (threadIdx.x == 0) part[(job * nbx + bx) * kSiaMax + i] = {re, im};
  }
}

// out[job * ostride + i] = sum over q < nq of part[job][q][i], i < ni.
__global__ __launch_bounds__(256) void k_sia_reduce(const cx<double> *part, int64_t nq, int32_t pstride,
                                                    int32_t ni, cx<double> *out, int64_t ostride) {
  __shared__ double lds[4];
  const int64_t job = blockIdx.x;
  for (int i = 0; i < ni; ++i) {
    double re = 0.0, im = 0.0;
    for (int64_t q = threadIdx.x; q < nq; q += kBlock) {
      const cx<double> p = part[(job * nq + q) * pstride + i];
      re += p.x;
      im += p.y;
    }
    re = block_sum(re, lds);
    im = block_sum(im, lds);
    if (threadIdx.x == 0) out[job * ostride + i] = {re, im};
  }
}

// V_w -= sum_{i < nd} h[job][i] V_i  (one Gram-Schmidt pass).
template <typename R>
__global__ __launch_bounds__(256) void k_sia_axpy(cx<R> *V, int64_t vstride, int64_t Z, int64_t nbx, int32_t w,
                                                  int32_t nd, const cx<double> *h, int64_t hstride) {
  const int64_t job = blockIdx.x / nbx, bx = blockIdx.x - job * nbx;
  const int64_t M = bx * kBlock + threadIdx.x;
  if (M >= Z) return;
  cx<R> *v = V + job * vstride;
  for (int e = 0; e < 4; ++e) {
    cx<R> acc = v[(int64_t)w * 4 * Z + e * Z + M];
    for (int i = 0; i < nd; ++i) {
      const cx<double> c = h[job * hstride + i];
      const cx<R> a = v[(int64_t)i * 4 * Z + e * Z + M];
      acc = csub(acc, cmul(cx<R>{(R)c.x, (R)c.y}, a));
    }
    v[(int64_t)w * 4 * Z + e * Z + M] = acc;
  }
}

// Whether the residual of Arnoldi column j is rounding noise, i.e. the Krylov space became
// invariant: its squared norm n2 against that of A v_j, sum_i |h_ij|^2 + n2 (both passes).
__host__ __device__ inline bool sia_breakdown(const cx<double> *h1, const cx<double> *h2, int nd, double n2,
                                              double rel2) {
  double tot = n2;
  for (int i = 0; i < nd; ++i) {
    const double re = h1[i].x + h2[i].x, im = h1[i].y + h2[i].y;
    tot += re * re + im * im;
  }
  return !(n2 > rel2 * tot) || !(n2 > 1e-300);
}

// V_w /= sqrt(Re nrm[job]), or V_w = 0 when the Krylov space became invariant.  h points at
// the first Gram-Schmidt pass of the column (the second follows at +hgap).
template <typename R>
__global__ __launch_bounds__(256) void k_sia_scale(cx<R> *V, int64_t vstride, int64_t Z, int64_t nbx, int32_t w,
                                                   const cx<double> *nrm, int64_t nstride, const cx<double> *h,
                                                   int32_t hgap, double rel2) {
  const int64_t job = blockIdx.x / nbx, bx = blockIdx.x - job * nbx;
  const int64_t M = bx * kBlock + threadIdx.x;
  if (M >= Z) return;
  const double n2 = nrm[job * nstride].x;
  const cx<double> *hj = h + job * nstride;
  const R s = sia_breakdown(hj, hj + hgap, w, n2, rel2) ? R(0) : (R)(1.0 / sqrt(n2));
  cx<R> *v = V + job * vstride + (int64_t)w * 4 * Z;
  for (int e = 0; e < 4; ++e) v[e * Z + M] = cscale(s, v[e * Z + M]);
}

// Partial Gram matrix of singlet amplitudes d_a = V_a(ab) - V_a(ba), pairs a <= b < m, one
// entry per wave: part[job][4 bx + wave][pair] = sum conj(d_a) d_b.
template <typename R>
__global__ __launch_bounds__(256) void k_sia_gram(const cx<R> *V, int64_t vstride, int64_t Z, int64_t nbx,
                                                  int32_t m, cx<double> *part, int32_t pstride) {
  const int64_t job = blockIdx.x / nbx, bx = blockIdx.x - job * nbx;
  const int64_t M = bx * kBlock + threadIdx.x;
  const bool live = M < Z;
  const cx<R> *v = V + job * vstride;
  cx<double> d[kSiaMax];
  for (int a = 0; a < m; ++a) {
    if (live) {
      const cx<R> p = v[(int64_t)a * 4 * Z + Z + M], q = v[(int64_t)a * 4 * Z + 2 * Z + M];
      d[a] = {(double)p.x - (double)q.x, (double)p.y - (double)q.y};
    } else {
      d[a] = {0.0, 0.0};
    }
  }
  const int wave = threadIdx.x >> 6;
  cx<double> *out = part + ((job * nbx + bx) * 4 + wave) * (int64_t)pstride;
  int pr = 0;
  for (int a = 0; a < m; ++a)
    for (int b = a; b < m; ++b, ++pr) {
      const double re = warp_sum(d[a].x * d[b].x + d[a].y * d[b].y);
      const double im = warp_sum(d[a].x * d[b].y - d[a].y * d[b].x);
      if ((threadIdx.x & 63) == 0) out[pr] = {re, im};
    }
}

// V_m = sum_{a < m} g[job][a] V_a, then V_0 = V_m (the normalised state for the next step).
template <typename R>
__global__ __launch_bounds__(256) void k_sia_combine(cx<R> *V, int64_t vstride, int64_t Z, int64_t nbx, int32_t m,
                                                     const cx<double> *g) {
  const int64_t job = blockIdx.x / nbx, bx = blockIdx.x - job * nbx;
  const int64_t M = bx * kBlock + threadIdx.x;
  if (M >= Z) return;
  cx<R> *v = V + job * vstride;
  for (int e = 0; e < 4; ++e) {
    cx<R> acc = {R(0), R(0)};
    for (int a = 0; a < m; ++a) {
      const cx<double> c = g[job * kSiaMax + a];
      acc = cadd(acc, cmul(cx<R>{(R)c.x, (R)c.y}, v[(int64_t)a * 4 * Z + e * Z + M]));
    }
    v[(int64_t)m * 4 * Z + e * Z + M] = acc;
  }
  for (int e = 0; e < 4; ++e) v[e * Z + M] = v[(int64_t)m * 4 * Z + e * Z + M];
}

// Small dense complex matrices (row-major n x n) for the Krylov-space algebra on the host.
using cplx = std::complex<double>;

static void small_matmul(const std::vector<cplx> &A, const std::vector<cplx> &B, std::vector<cplx> &C, int n) {
  C.assign((size_t)n * n, cplx(0.0, 0.0));
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) {
      const cplx a = A[(size_t)i * n + k];
      if (a == cplx(0.0, 0.0)) continue;
      for (int j = 0; j < n; ++j) C[(size_t)i * n + j] += a * B[(size_t)k * n + j];
    }
}

// exp(A) by scaling and squaring with a degree-16 Taylor polynomial evaluated at A / 2^s,
// ||A / 2^s||_1 <= 1/4 (remainder below 1e-24 relative).
static void small_expm(const std::vector<cplx> &A, std::vector<cplx> &E, int n) {
  double nrm = 0.0;
  for (int j = 0; j < n; ++j) {
    double c = 0.0;
    for (int i = 0; i < n; ++i) c += std::abs(A[(size_t)i * n + j]);
    nrm = std::max(nrm, c);
  }
  int s = 0;
  while (nrm > 0.25 && s < 200) {
    nrm *= 0.5;
    ++s;
  }
  const double sc = std::ldexp(1.0, -s);
  std::vector<cplx> As(A.size()), T((size_t)n * n, cplx(0.0, 0.0)), P;
  for (size_t i = 0; i < A.size(); ++i) As[i] = A[i] * sc;
  for (int i = 0; i < n; ++i) T[(size_t)i * n + i] = 1.0;
  for (int k = 16; k >= 1; --k) {   // T = I + As T / k
    small_matmul(As, T, P, n);
    for (size_t i = 0; i < P.size(); ++i) P[i] /= (double)k;
    for (int i = 0; i < n; ++i) P[(size_t)i * n + i] += 1.0;
    T.swap(P);
  }
  for (int q = 0; q < s; ++q) {
    small_matmul(T, T, P, n);
    T.swap(P);
  }
  E.swap(T);
}

struct SiaJob {
  double t = 0.0, beta = 1.0, phi = 0.0, dt = 0.0;
  int64_t steps = 0;
  bool done = false, failed = false;
};
constexpr int64_t kSiaMaxSteps = 1000000;   // per job; more means the step control has failed

// One Arnoldi step of one job on the host: step length from the error estimate, the in-step
// yield by Van Loan's block exponential, and the coefficients of the next normalised state.
static void sia_host_step(const cplx *blk, int m, double T, double kS, double kT, double tol, double rel2,
                          SiaJob &jb, cplx *g) {
  for (int a = 0; a < kSiaMax; ++a) g[a] = 0.0;
  if (jb.done) {
    g[0] = 1.0;
    return;
  }
  // Hessenberg matrix: H[i][j] = both Gram-Schmidt passes; H[j+1][j] = norm of the residual.
  std::vector<cplx> X((size_t)m * m, cplx(0.0, 0.0));
  const cplx *nrm = blk + 2 * m * (m + 1);
  double hlast = 0.0;
  for (int j = 0; j < m; ++j) {
    const cplx *h1 = blk + (j * 2) * (m + 1), *h2 = blk + (j * 2 + 1) * (m + 1);
    for (int i = 0; i <= j; ++i) X[(size_t)i * m + j] = cplx(0.0, -1.0) * (h1[i] + h2[i]);
    // the same breakdown decision as the device's normalisation
    const bool bd = sia_breakdown(reinterpret_cast<const cx<double> *>(h1), reinterpret_cast<const cx<double> *>(h2),
                                  j + 1, nrm[j].real(), rel2);
    const double hn = bd ? 0.0 : std::sqrt(nrm[j].real());
    if (j + 1 < m) X[(size_t)(j + 1) * m + j] = cplx(0.0, -hn);
    else hlast = hn;
  }
  // S[a][b] = <P_S v_a | P_S v_b> = (1/2) sum conj(d_a) d_b
  std::vector<cplx> S((size_t)m * m);
  const cplx *gr = nrm + m;
  for (int a = 0, pr = 0; a < m; ++a)
    for (int b = a; b < m; ++b, ++pr) {
      S[(size_t)a * m + b] = 0.5 * gr[pr];
      S[(size_t)b * m + a] = std::conj(0.5 * gr[pr]);
    }
  double dt = std::min(T - jb.t, jb.dt > 0.0 ? 1.5 * jb.dt : T - jb.t);
  std::vector<cplx> E, Xs((size_t)m * m);
  for (int tries = 0;; ++tries) {
    for (size_t i = 0; i < X.size(); ++i) Xs[i] = X[i] * dt;
    small_expm(Xs, E, m);
    const double err = hlast * std::abs(E[(size_t)(m - 1) * m + 0]);
    if (err <= tol) break;
    if (tries >= 60 || !std::isfinite(err)) {   // no admissible step: report instead of crawling
      jb.failed = true;
      jb.done = true;
      g[0] = 1.0;
      return;
    }
    dt *= 0.6;
  }
  if (T - jb.t - dt < 1e-14 * T) dt = T - jb.t;
  // Van Loan: exp([[-Xd^H, S], [0, Xd]] dt) = [[., G1], [0, F3]], int_0^dt e^{Xd^H s} S e^{Xd s} ds
  // = F3^H G1, with Xd = X - (kT/2) I carrying the scalar decay of the population.
  const int n2 = 2 * m;
  std::vector<cplx> C((size_t)n2 * n2, cplx(0.0, 0.0)), F;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      const cplx xd = X[(size_t)i * m + j] - (i == j ? 0.5 * kT : 0.0);
      const cplx xdh = std::conj(X[(size_t)j * m + i] - (i == j ? 0.5 * kT : 0.0));
      C[(size_t)i * n2 + j] = -xdh * dt;
      C[(size_t)i * n2 + m + j] = S[(size_t)i * m + j] * dt;
      C[(size_t)(m + i) * n2 + m + j] = xd * dt;
    }
  small_expm(C, F, n2);
  cplx q = 0.0;
  for (int a = 0; a < m; ++a) q += std::conj(F[(size_t)(m + a) * n2 + m]) * F[(size_t)a * n2 + m];
  jb.phi += kS * jb.beta * jb.beta * std::exp(-kT * jb.t) * q.real();
  double cn = 0.0;
  for (int a = 0; a < m; ++a) cn += std::norm(E[(size_t)a * m]);
  cn = std::sqrt(cn);
  for (int a = 0; a < m; ++a) g[a] = cn > 0.0 ? E[(size_t)a * m] / cn : cplx(a == 0 ? 1.0 : 0.0, 0.0);
  jb.beta *= cn;
  jb.t += dt;
  jb.dt = dt;
  if (jb.t >= T * (1.0 - 1e-14)) jb.done = true;
  if (++jb.steps >= kSiaMaxSteps && !jb.done) {
    jb.failed = true;
    jb.done = true;
  }
}

template <typename R>
static int sia_system(const SystemSpec &spec, const double *B, int nB, const double *angles_dev, int64_t M,
                      const Opts &op, double *phi_out, hipStream_t st) {
  const int m = op.krylov;
  const double tol = op.tol_set ? op.tol : (op.precision == 64 ? 1e-13 : 1e-8);
  // A residual below 1e-14 (FP64) or 1e-6 (FP32) of |A v_j| is rounding noise: the Krylov space
  // is invariant and the column ends the space.
  const double rel2 = op.precision == 64 ? 1e-28 : 1e-12;
  const int64_t Z = spec.Z;
  const int N = spec.N();
  const int64_t nbx = (Z + kBlock - 1) / kBlock;
  const int64_t total_jobs = (int64_t)nB * M;
  if (total_jobs == 0) return RP_OK;
  const int64_t vstride = (int64_t)(m + 1) * 4 * Z;
  const int npair = m * (m + 1) / 2;
  const int64_t small = 2 * m * (m + 1) + m + npair;   // complex entries per job copied to the host
  const int64_t per_job = vstride * (int64_t)sizeof(cx<R>) + nbx * kSiaMax * 16 + nbx * 4 * npair * 16 +
                          small * 16 + kSiaMax * 16 + 64;
  int64_t budget = op.workspace;
  if (budget <= 0) {
    size_t fr = 0, tot = 0;
    HIPCHK(hipMemGetInfo(&fr, &tot));
    budget = (int64_t)(fr / 2);
  }
  int64_t chunk = std::min<int64_t>({total_jobs, budget / per_job, (int64_t)256, (((int64_t)1) << 24) / nbx});
  if (chunk < 1) return fail(RP_ENOMEM, "workspace too small for one wavepacket");
  struct Buf {
    void *p = nullptr;
    ~Buf() { if (p) (void)hipFree(p); }
  };
  Buf bV, bPd, bPg, bSm, bG, bOm, bTab, bJs;
  auto alloc = [&](Buf &b, size_t bytes) -> int {
    if (hipMalloc(&b.p, std::max<size_t>(bytes, 16)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(RP_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    return RP_OK;
  };
  int rc;
  if ((rc = alloc(bV, (size_t)chunk * vstride * sizeof(cx<R>)))) return rc;
  if ((rc = alloc(bPd, (size_t)chunk * nbx * kSiaMax * 16))) return rc;
  if ((rc = alloc(bPg, (size_t)chunk * nbx * 4 * npair * 16))) return rc;
  if ((rc = alloc(bSm, (size_t)chunk * small * 16))) return rc;
  if ((rc = alloc(bG, (size_t)chunk * kSiaMax * 16))) return rc;
  if ((rc = alloc(bOm, (size_t)chunk * 8))) return rc;
  if ((rc = alloc(bJs, (size_t)total_jobs * 4))) return rc;
  if ((rc = alloc(bTab, (size_t)std::max<int64_t>(M, 1) * std::max(N, 1) * (RP_MAX_TWO_I + 1) * sizeof(cx<double>))))
    return rc;
  std::vector<int32_t> job_sample(total_jobs);
  for (int64_t j = 0; j < total_jobs; ++j) job_sample[j] = (int32_t)(j % M);
  HIPCHK(hipMemcpyAsync(bJs.p, job_sample.data(), total_jobs * 4, hipMemcpyHostToDevice, st));
  if (N > 0) {
    CohArgs ca;
    std::memset(&ca, 0, sizeof(ca));
    ca.angles = angles_dev;
    ca.tab = (cx<double> *)bTab.p;
    ca.M = M;
    ca.N = N;
    ca.mode = op.init_mode;
    for (int k = 0; k < N; ++k) {
      ca.two_I[k] = spec.two_I[k];
      ca.perm[k] = spec.perm[k];
    }
    hipLaunchKernelGGL(k_coherent, dim3(grid1(M * N)), dim3(256), 0, st, ca);
    HIPCHK(hipGetLastError());
  }
  const SysArgs<R> sa = make_sysargs<R>(spec);
  cx<R> *V = (cx<R> *)bV.p;
  cx<double> *Pd = (cx<double> *)bPd.p, *Pg = (cx<double> *)bPg.p, *Sm = (cx<double> *)bSm.p;
  std::vector<cplx> hsmall((size_t)chunk * small), hg((size_t)chunk * kSiaMax);
  const int nth = std::max(1, (int)std::thread::hardware_concurrency());
  for (int64_t j0 = 0; j0 < total_jobs; j0 += chunk) {
    const int64_t nj = std::min(chunk, total_jobs - j0);
    const unsigned grid = (unsigned)(nj * nbx);
    std::vector<double> om(nj);
    for (int64_t j = 0; j < nj; ++j) om[j] = spec.gamma * B[(j0 + j) / M];
    HIPCHK(hipMemcpyAsync(bOm.p, om.data(), nj * 8, hipMemcpyHostToDevice, st));
    {
      InitArgs<R> ia;
      std::memset(&ia, 0, sizeof(ia));
      ia.psi = V;
      ia.vstride = vstride;
      ia.tab = (const cx<double> *)bTab.p;
      ia.job_sample = (const int32_t *)bJs.p + j0;
      ia.Z = Z;
      ia.nbx = nbx;
      ia.njobs = (int32_t)nj;
      ia.N = N;
      for (int k = 0; k < N; ++k) {
        ia.stride[k] = sa.stride[k];
        ia.d[k] = sa.d[k];
      }
      if (N == 0) {
        ia.stride[0] = 1;
        ia.d[0] = 1;
      }
      ia.tiles = (int64_t)grid;
      hipLaunchKernelGGL((k_init<R, false>), dim3(grid), dim3(kBlock), 0, st, ia);
      HIPCHK(hipGetLastError());
    }
    std::vector<SiaJob> jobs(nj);
    for (;;) {
      bool all_done = true;
      for (auto &jb : jobs) all_done = all_done && jb.done;
      if (all_done) break;
      for (int j = 0; j < m; ++j) {
        const int w = j + 1;
        hipLaunchKernelGGL(k_sia_apply<R>, dim3(grid), dim3(kBlock), 0, st, sa, V + (int64_t)j * 4 * Z,
                           V + (int64_t)w * 4 * Z, vstride, nbx, (int32_t)nj, (const double *)bOm.p);
        for (int pass = 0; pass < 2; ++pass) {   // classical Gram-Schmidt, twice
          cx<double> *h = Sm + (j * 2 + pass) * (m + 1);
          hipLaunchKernelGGL(k_sia_dot<R>, dim3(grid), dim3(kBlock), 0, st, V, vstride, Z, nbx, (int32_t)nj, w, 0,
                             j + 1, Pd);
          hipLaunchKernelGGL(k_sia_reduce, dim3((unsigned)nj), dim3(kBlock), 0, st, Pd, nbx, kSiaMax, j + 1, h,
                             small);
          hipLaunchKernelGGL(k_sia_axpy<R>, dim3(grid), dim3(kBlock), 0, st, V, vstride, Z, nbx, w, j + 1, h, small);
        }
        cx<double> *nr = Sm + 2 * m * (m + 1) + j;
        hipLaunchKernelGGL(k_sia_dot<R>, dim3(grid), dim3(kBlock), 0, st, V, vstride, Z, nbx, (int32_t)nj, w, w, 1,
                           Pd);
        hipLaunchKernelGGL(k_sia_reduce, dim3((unsigned)nj), dim3(kBlock), 0, st, Pd, nbx, kSiaMax, 1, nr, small);
        hipLaunchKernelGGL(k_sia_scale<R>, dim3(grid), dim3(kBlock), 0, st, V, vstride, Z, nbx, w, nr, small,
                           Sm + (j * 2) * (m + 1), m + 1, rel2);
      }
      hipLaunchKernelGGL(k_sia_gram<R>, dim3(grid), dim3(kBlock), 0, st, V, vstride, Z, nbx, m, Pg, npair);
      hipLaunchKernelGGL(k_sia_reduce, dim3((unsigned)nj), dim3(kBlock), 0, st, Pg, nbx * 4, npair, npair,
                         Sm + 2 * m * (m + 1) + m, small);
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(hsmall.data(), Sm, (size_t)nj * small * 16, hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      std::vector<std::thread> th;
      for (int q = 0; q < std::min<int64_t>(nth, nj); ++q)
        th.emplace_back([&, q]() {
          for (int64_t j = q; j < nj; j += nth)
            sia_host_step(&hsmall[(size_t)j * small], m, spec.T, spec.kS, spec.kT, tol, rel2, jobs[j],
                          &hg[(size_t)j * kSiaMax]);
        });
      for (auto &x : th) x.join();
      for (auto &jb : jobs)
        if (jb.failed || !std::isfinite(jb.phi) || !std::isfinite(jb.beta))
          return fail(RP_ENOTCONV, "Arnoldi step control found no admissible step");
      HIPCHK(hipMemcpyAsync(bG.p, hg.data(), (size_t)nj * kSiaMax * 16, hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(k_sia_combine<R>, dim3(grid), dim3(kBlock), 0, st, V, vstride, Z, nbx, m,
                         (const cx<double> *)bG.p);
      HIPCHK(hipGetLastError());
    }
    std::vector<double> ph(nj);
    for (int64_t j = 0; j < nj; ++j) ph[j] = jobs[j].phi;
    if (op.flags & RP_FLAG_PROFILE)
      for (auto &jb : jobs) {
        g_prof.terms += (double)jb.steps * m;      // applications of A per job, summed
        g_prof.quad_launches += (double)jb.steps;  // Arnoldi steps, summed over jobs
      }
    HIPCHK(hipMemcpyAsync(phi_out + j0, ph.data(), nj * 8, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  return RP_OK;
}

// Argument checks shared by rp_propagate and rp_propagate_static (RP_OK, or an error code; *empty
// is set when there is nothing to do).
static int check_propagate(const rp_system *sys, int32_t n_sys, const double *B_mT, int32_t nB, const double *angles,
                           int64_t M, const rp_opts *opts, double *phi, double *ps_t, Opts &op, bool &empty) {
  empty = false;
  if (n_sys < 0 || nB < 0 || M < 0) return fail(RP_EINVAL, "negative count");
  if (n_sys == 0 || nB == 0 || M == 0) {
    empty = true;
    return RP_OK;
  }
  if (!sys || !B_mT || !phi) return fail(RP_EINVAL, "null pointer");
  if (M > (int64_t)1 << 31) return fail(RP_EINVAL, "M too large");
  int rc = read_opts(opts, op);
  if (rc) return rc;
  if (ps_t && (op.flags & RP_FLAG_ARNOLDI))
    return fail(RP_ENOTIMPL, "trajectory output needs the Chebyshev steps (not RP_FLAG_ARNOLDI)");
  if (ps_t && op.ps_len < 1) return fail(RP_EINVAL, "ps_t needs opts->ps_t_len >= 1");
  if (ps_t && (double)n_sys * nB * (double)M * (double)op.ps_len > 0x1p38) return fail(RP_EINVAL, "ps_t too large");
  for (int i = 0; i < n_sys; ++i) {
    rc = validate_system(&sys[i]);
    if (rc) return rc;
    if (sys[i].n_nuc[0] + sys[i].n_nuc[1] > 0 && !angles) return fail(RP_EINVAL, "null angles");
  }
  for (int64_t i = 0; i < (int64_t)n_sys * nB; ++i)
    if (!std::isfinite(B_mT[i])) return fail(RP_EINVAL, "non-finite field");
  return RP_OK;
}

extern "C" int rp_propagate(const rp_system *sys, int32_t n_sys, const double *B_mT, int32_t nB,
                            const double *angles, int64_t M, const rp_opts *opts, double *phi, double *ps_t,
                            void *hip_stream) {
  g_err.clear();
  Opts op;
  bool empty = false;
  int rc = check_propagate(sys, n_sys, B_mT, nB, angles, M, opts, phi, ps_t, op, empty);
  if (rc || empty) return rc;
  hipStream_t st = (hipStream_t)hip_stream;
  // The legacy default stream cannot be captured into a graph: run the call on a blocking
  // stream of its own (implicitly ordered with the default stream; the call synchronises
  // before returning, so its results are ready either way).
  struct OwnStream {
    hipStream_t s = nullptr;
    ~OwnStream() { if (s) { (void)hipStreamSynchronize(s); (void)hipStreamDestroy(s); } }
  } own;
  if (!st) {
    HIPCHK(hipStreamCreate(&own.s));
    st = own.s;
  }
  if (op.flags & RP_FLAG_ARNOLDI) {   // short-iterative Arnoldi, one system at a time
    if (op.flags & RP_FLAG_PROFILE) g_prof = Profile();
    int64_t aoff = 0;
    for (int i = 0; i < n_sys; ++i) {
      const rp_system *s = &sys[i];
      const int N = s->n_nuc[0] + s->n_nuc[1];
      SystemSpec spec = tile_order(make_spec(s->n_nuc[0], s->n_nuc[1], s->two_I, s->a_mT, s->J_mT, s->kS, s->kT,
                                             s->T_us, gamma_of(s)),
                                   (op.flags & RP_FLAG_AXES_HIGH_FIRST) != 0);
      const double *ang = angles ? angles + aoff : nullptr;
      double *out = phi + (int64_t)i * nB * M;
      rc = op.precision == 64 ? sia_system<double>(spec, B_mT + (int64_t)i * nB, nB, ang, M, op, out, st)
                              : sia_system<float>(spec, B_mT + (int64_t)i * nB, nB, ang, M, op, out, st);
      if (rc) return rc;
      aoff += M * N * 2;
    }
    return RP_OK;
  }
  EventLog log;
  log.on = (op.flags & RP_FLAG_PROFILE) != 0;
  if (log.on) g_prof = Profile();
  hipEvent_t t0 = log.mark(st);
  rc = op.precision == 64
           ? propagate_chebyshev<double>(sys, n_sys, B_mT, nB, angles, M, op, phi, ps_t, st, log, nullptr, 0)
           : propagate_chebyshev<float>(sys, n_sys, B_mT, nB, angles, M, op, phi, ps_t, st, log, nullptr, 0);
  if (rc) return rc;
  if (log.on) {
    hipEvent_t t1 = nullptr;
    if (hipEventCreate(&t1) == hipSuccess) {
      (void)hipEventRecord(t1, st);
      (void)hipEventSynchronize(t1);
      float ms = 0.f;
      if (t0 && hipEventElapsedTime(&ms, t0, t1) == hipSuccess) g_prof.total_ms = ms;
      (void)hipEventDestroy(t1);
    }
    // the first event (t0) is not part of a pair: drop it before resolving pairs
    if (!log.ev.empty()) {
      (void)hipEventDestroy(log.ev.front());
      log.ev.erase(log.ev.begin());
    }
    log.resolve(g_prof);
  }
  return RP_OK;
}

// ----------------------------------------------------------------------------- without allocation
// The workspace of rp_propagate_static: a file-scope device array that every GPU the library
// runs on holds (its own copy, at its own address) until the process ends.  In host code the
// name `scratch` is only a host-side stand-in: kernels and copies get the device address that
// hipGetSymbolAddress reports for the current device, looked up once per device.
constexpr int64_t kScratchBytes = (int64_t)RP_STATIC_SCRATCH_MB << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static char *g_scratch_ptr[64];   // device address of `scratch` per device id (null until looked up)

static int scratch_address(char **out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(RP_EDEVICE, "device id out of range for the static scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(RP_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = (char *)p;
  }
  *out = g_scratch_ptr[dev];
  return RP_OK;
}

extern "C" int rp_propagate_static(const rp_system *sys, int32_t n_sys, const double *B_mT, int32_t nB,
                                   const double *angles, int64_t M, const rp_opts *opts, double *phi, double *ps_t,
                                   void *hip_stream) {
  g_err.clear();
  Opts op;
  bool empty = false;
  int rc = check_propagate(sys, n_sys, B_mT, nB, angles, M, opts, phi, ps_t, op, empty);
  if (rc || empty) return rc;
  if (op.flags & (RP_FLAG_ARNOLDI | RP_FLAG_PROFILE))
    return fail(RP_ENOTIMPL, "rp_propagate_static: RP_FLAG_ARNOLDI and RP_FLAG_PROFILE need rp_propagate");
  if (op.workspace > 0 && op.workspace < kScratchBytes)
    return fail(RP_EINVAL, "rp_propagate_static: workspace_bytes must be 0 (the static area is used whole)");
  char *base = nullptr;
  if ((rc = scratch_address(&base))) return rc;
  EventLog log;   // off: no events
  hipStream_t st = (hipStream_t)hip_stream;
  return op.precision == 64
             ? propagate_chebyshev<double>(sys, n_sys, B_mT, nB, angles, M, op, phi, ps_t, st, log, base, kScratchBytes)
             : propagate_chebyshev<float>(sys, n_sys, B_mT, nB, angles, M, op, phi, ps_t, st, log, base, kScratchBytes);
}

extern "C" int rp_profile_last(double *out, int32_t n) {
  if (!out || n < 0) return fail(RP_EINVAL, "bad profile buffer");
  const double v[8] = {g_prof.term_ms, g_prof.term_launches, g_prof.elems,
                       g_prof.elems > 0 ? g_prof.bytes / g_prof.elems : 0.0,
                       g_prof.quad_ms, g_prof.quad_launches, g_prof.total_ms, g_prof.terms};
  const int m = n < 8 ? n : 8;
  for (int i = 0; i < m; ++i) out[i] = v[i];
  return m;
}

extern "C" int rp_cv_beta(const double *phi, const double *g, int32_t nB, int64_t M, double *beta,
                          void *hip_stream) {
  if (nB < 0 || M < 1) return fail(RP_EINVAL, "bad sizes");
  if (nB == 0) return RP_OK;
  if (!phi || !g || !beta) return fail(RP_EINVAL, "null pointer");
  BetaArgs a{phi, g, beta, M};
  hipLaunchKernelGGL(k_beta, dim3(nB), dim3(256), 0, (hipStream_t)hip_stream, a);
  HIPCHK(hipGetLastError());
  return RP_OK;
}

extern "C" int rp_combine(const double *mean_a, const double *err_a, const double *mean_b, const double *err_b,
                          int32_t nB, double *mean, double *err, void *hip_stream) {
  g_err.clear();
  if (nB < 0) return fail(RP_EINVAL, "negative count");
  if (nB == 0) return RP_OK;
  if (!mean_a || !err_a || !mean_b || !err_b || !mean || !err) return fail(RP_EINVAL, "null pointer");
  hipLaunchKernelGGL(k_combine, dim3(grid1(nB)), dim3(256), 0, (hipStream_t)hip_stream, mean_a, err_a, mean_b, err_b,
                     nB, mean, err);
  HIPCHK(hipGetLastError());
  return RP_OK;
}

__global__ __launch_bounds__(256) void k_group_mean(const double *phi, int64_t n_out, int64_t group, double *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_out) return;
  const double *p = phi + i * group;
  double t = 0.0;
  for (int64_t j = 0; j < group; ++j) t += p[j];
  out[i] = t / (double)group;
}

extern "C" int rp_group_mean(const double *phi, int32_t nB, int64_t M, int64_t group, double *out,
                             void *hip_stream) {
  if (nB < 0 || M < 0) return fail(RP_EINVAL, "negative count");
  if (group < 1 || M % group != 0) return fail(RP_EINVAL, "group must be >= 1 and divide M");
  if (nB == 0 || M == 0) return RP_OK;
  if (!phi || !out) return fail(RP_EINVAL, "null pointer");
  const int64_t n_out = (int64_t)nB * (M / group);
  if (n_out > ((int64_t)1 << 38)) return fail(RP_EINVAL, "too many groups");
  hipLaunchKernelGGL(k_group_mean, dim3(grid1(n_out)), dim3(256), 0, (hipStream_t)hip_stream, phi, n_out, group,
                     out);
  HIPCHK(hipGetLastError());
  return RP_OK;
}

extern "C" int rp_yield(const double *phi, int32_t nB, int64_t M, const double *cv_g, const double *cv_mu,
                        const double *cv_beta, const double *cv_mu_err, double *mean, double *stderr_,
                        void *hip_stream) {
  if (nB < 0 || M < 0) return fail(RP_EINVAL, "negative count");
  if (nB == 0) return RP_OK;
  if (M == 0) return fail(RP_EINVAL, "M must be >= 1");
  if (!phi || !mean || !stderr_) return fail(RP_EINVAL, "null pointer");
  if (cv_g && (!cv_mu || !cv_beta)) return fail(RP_EINVAL, "control variate needs mu and beta");
  StatArgs a{phi, cv_g, cv_mu, cv_beta, cv_mu_err, mean, stderr_, M};
  hipLaunchKernelGGL(k_stats, dim3(nB), dim3(256), 0, (hipStream_t)hip_stream, a);
  HIPCHK(hipGetLastError());
  return RP_OK;
}
