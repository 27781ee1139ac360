// Device-side data structures and kernels of librp (gfx950, wave64).
//
// Wavepacket layout in HBM: one job (system, field, sample) owns a contiguous
// vector of 4Z complex numbers stored as four planes, element index  e Z + M,
// where e = 2 b1 + b2 enumerates the electron product states (aa, ab, ba, bb)
// with b = 1 for beta, and M = sum_k n_k stride_k is the mixed-radix nuclear
// index with digit n_k = I_k - m_k (first nucleus fastest).  Each complex number
// is interleaved (re, im).  Planes make every partner read along a slow nuclear
// axis a unit-stride load of exactly the two components it needs.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "rp.h"

namespace rp {

constexpr int kBlock = 256;   // threads per workgroup: one nuclear index M per thread
constexpr int kQuadChunk = 16;

template <typename R>
struct cx {
  R x, y;
};

// Loads and stores with the non-temporal hint (ON = true), for data touched once per launch,
// so that it does not displace from the caches the data that is re-read: the partner tiles of
// phi_n within a launch, and (when the chunk fits the Infinity Cache) phi_{n+1} for the next.
template <typename R>
using cxv = R __attribute__((ext_vector_type(2)));
template <bool ON, typename R>
__device__ __forceinline__ cx<R> ld_nt(const cx<R> *p) {
  if constexpr (ON) {
    const cxv<R> v = __builtin_nontemporal_load(reinterpret_cast<const cxv<R> *>(p));
    return {v.x, v.y};
  } else {
    return *p;
  }
}
template <bool ON, typename R>
__device__ __forceinline__ void st_nt(cx<R> *p, cx<R> v) {
  if constexpr (ON) {
    cxv<R> t;
    t.x = v.x;
    t.y = v.y;
    __builtin_nontemporal_store(t, reinterpret_cast<cxv<R> *>(p));
  } else {
    *p = v;
  }
}

// Per-system constants in the kernel-argument segment (uniform across the grid).
template <typename R>
struct SysArgs {
  int32_t N, N1, all_half, nhalf;   // nhalf: leading spin-1/2 nuclei (strides 2^k)
  int32_t tiled, pad0, pad1, pad2;  // tiled: k_cheb_tile applies (nhalf == N, or nhalf >= 8)
  int64_t Z;
  R J;       // exchange (rad/us): diagonal +-J/2, ab<->ba coupling J
  R beta;    // coefficient of i*beta*P_S in the kernel operator
  int32_t stride[RP_MAX_NUCLEI];
  int32_t d[RP_MAX_NUCLEI];
  int32_t shift[RP_MAX_NUCLEI];        // log2(stride) for the leading spin-1/2 nuclei
  int32_t rad[RP_MAX_NUCLEI];          // radical (0, 1) of each nucleus
  R a[RP_MAX_NUCLEI];                  // a_k (rad/us), for the diagonal sum a_k m_k
  R f[RP_MAX_NUCLEI][RP_MAX_TWO_I];    // (a_k/2) sqrt(I(I+1) - m(m-1)), link between digits n, n+1
};

// Per-field constants of one Chebyshev step.
template <typename R>
struct FieldDev {
  R omega;        // gamma B
  R c_re, c_im;   // shift of the kernel operator (includes -i dk/2 when P_T is dissipative)
  R s1, s2;       // 1/r and 2/r
};

// One job (system, field, sample) of a chunk in the job queue of the tiled kernels.  The jobs of a
// chunk are laid out one after another: wavepacket vectors at `vec` (4Z complex numbers),
// singlet amplitudes at `amp` within each term slab (Z), workgroups (256-index tiles) from `blk`.
struct QJob {
  int32_t sys;             // index into the per-call system table
  int32_t field;           // index into the per-call field tables (system-major)
  int32_t nbx;             // tiles of this job
  int32_t pad;
  int64_t Z;               // nuclear states
  int64_t vec, amp, blk;   // offsets within the chunk (complex numbers, complex numbers, tiles)
  int64_t tab;             // row of the job's first nucleus in the coherent-state table
};

template <typename R>
struct TermArgs {
  const cx<R> *phin;       // phi_n, [jobs][4Z]
  cx<R> *phio;             // in: phi_{n-1}; out: phi_{n+1} (same storage)
  cx<R> *acc;              // running sum_n a_n phi_n
  cx<R> *dnext;            // singlet amplitudes of phi_{n+1}: [jobs][Z]
  cx<R> *dfirst;           // first term only: singlet amplitudes of phi_0
  const FieldDev<R> *fields;
  const cx<R> *coef;       // [fields][n_terms]
  const int32_t *job_field;
  double *part_norm;       // first term only: [tiles]
  // Job queue (several systems in one launch): tile -> job, job descriptors, system table.
  const int32_t *tile_job;
  const QJob *jobs;
  const SysArgs<R> *systab;
  int64_t nbx;             // tiles per job when every job of the launch has the same system
  int64_t tiles;           // tiles of the launch
  int32_t njobs;
  int32_t n;               // producing phi_{n+1}
  int32_t n_terms;
  int32_t remap;           // 1: each XCD takes a contiguous range of workgroups (see xcd_remap)
};

template <typename R>
struct QuadArgs {
  const cx<R> *d;          // [n_terms][slab]
  int64_t slab;            // elements per term slab (sum of Z over the chunk's jobs)
  const R *ell;            // [fields][n_terms][rank_pad]
  const int32_t *job_field;
  double *part;            // [tiles][2]: quadratic form, |d_0|^2/2
  const int32_t *tile_job; // job queue (several systems): as in TermArgs
  const QJob *jobs;
  int64_t Z;
  int64_t nbx;
  int64_t tiles;
  int32_t njobs;
  int32_t n_terms;
  int32_t rank_pad;
  int32_t remap;
};

struct FinArgs {
  const double *part_q;    // [tiles][2]
  const double *part_norm; // [tiles]
  double *phi;             // [jobs] accumulated yields of this chunk
  double *prev_norm;       // [jobs]
  int *flag;
  const int32_t *job_field;
  const double *dt;        // [fields]
  int32_t *stepc;          // [jobs] steps finalised so far (read, then incremented)
  const QJob *jobs;        // job queue (several systems), or null: nbx tiles per job
  const int32_t *slots;    // job queue: slot of each workgroup (occupied slots), or null
  const double *sys_k;     // job queue: [systems][2] = (kS, k_min)
  int64_t nbx;
  int32_t njobs;
  int32_t pad;
  double kS, kmin, rtol;
  double *ps_t;            // singlet population at step starts, [outputs][ps_len], or null
  const int64_t *dst;      // [jobs] output index of each job
  int64_t ps_len;
};

// ---------------------------------------------------------------- LDS-resident propagation
// Small systems (Z <= kResMax32 for complex FP32, kResMax64 for FP64): one workgroup per job
// runs the whole propagation with the wavepacket in LDS; jobs of several systems, fields and
// samples share one launch.
constexpr int kResMax32 = 1024;
constexpr int kResMax64 = 512;
constexpr int kResRank = 32;   // quadrature columns held in registers per thread

template <typename R>
struct ResSys {
  SysArgs<R> sa;
  int64_t tab_off;     // offset (in coherent-table rows of RP_MAX_TWO_I+1) of this system's samples
  double kS, kmin, rtol;
};

template <typename R>
struct ResField {
  FieldDev<R> fd;
  double dt;
  int64_t coef_off;    // into the coefficient array (n_terms entries)
  int64_t ell_off;     // into the quadrature factor array (n_terms x kResRank entries)
  int32_t n_steps, n_terms;
};

struct ResJob {
  int32_t sys, field, sample, pad;
  int64_t out;         // index into phi
};

template <typename R>
struct ResArgs {
  const ResSys<R> *sys;
  const ResField<R> *fields;
  const ResJob *jobs;
  const cx<R> *coef;
  const R *ell;
  const cx<double> *tab;
  double *phi;
  int *flag;
  int64_t njobs;
};

}  // namespace rp
