/*
 * librp -- spin-coherent-state Monte Carlo singlet yields of radical pairs on MI355X.
 *
 * Method: A. M. Lewis, T. P. Fay, D. E. Manolopoulos, "An efficient quantum
 * mechanical method for radical pair recombination reactions" (arXiv:1612.09517).
 * The ensemble singlet yield Phi_S = k_S int P_S(t) dt (Eq. 20) is estimated by
 * averaging single-wavepacket yields phi_S(Omega) (Eq. 22) over wavepackets
 * |S> (x) |Omega_1> (x) ... (x) |Omega_N> whose nuclear spin coherent states
 * (Eq. 15) point in directions sampled uniformly on each sphere (Eq. 18).
 *
 * Conventions shared by every entry point
 *   - Units: hyperfine couplings, exchange and fields in mT (converted with
 *     gamma to rad/us); rate constants k_S, k_T in 1/us; times in us.
 *   - Hamiltonian (Eq. 1): H = omega (S1z + S2z) + sum_k a_k I_k.S_i(k) + 2 J S1.S2
 *     with omega = gamma B along z (B < 0 reverses the field; single-wavepacket yields
 *     then differ, the ensemble yield is even in B), no nuclear
 *     Zeeman terms, hbar = 1.  Recombination by the Haberkorn operator
 *     K = k_S/2 P_S + k_T/2 P_T (Eq. 2-4); wavepackets evolve by
 *     exp(-iHt - Kt) (Eq. 13).
 *   - Nuclei are listed radical 1 first, then radical 2.  Spin quantum numbers
 *     are given as two_I = 2I (1 = spin-1/2, 2 = spin-1, ... at most 4).
 *   - Device pointers are HIP device allocations on the current device; host
 *     pointers are ordinary CPU memory.  The caller owns every buffer.
 *   - All work is enqueued on the given HIP stream (NULL = default stream).
 *     rp_sample and rp_yield return without waiting; rp_propagate waits for
 *     its own work to finish before it returns (it checks a convergence
 *     flag), so its outputs are ready on return.
 *   - Errors: every entry point returns RP_OK (0) or a negative code.
 *     Argument errors are detected before any device work is enqueued.
 *     rp_last_error() gives a message for the most recent failure on the
 *     calling thread.  The library never aborts the process.
 */
#ifndef RP_H
#define RP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  RP_OK = 0,
  RP_EINVAL = -1,   /* bad sizes, null pointers, negative rates, T <= 0, spin or nucleus limits */
  RP_ENOMEM = -2,   /* device workspace could not be allocated */
  RP_EDEVICE = -3,  /* a HIP call failed */
  RP_ENOTCONV = -4, /* wavepacket norm grew or became NaN: spectral bound violated */
  RP_ENOTIMPL = -5  /* option not implemented */
};

#define RP_MAX_NUCLEI 40
#define RP_MAX_TWO_I 4

/* One radical pair (Sec. II).  Read only during a call; arrays are host memory. */
typedef struct rp_system {
  int32_t n_nuc[2];      /* N1, N2: nuclei on radical 1 and radical 2 (N1+N2 <= RP_MAX_NUCLEI) */
  const int32_t *two_I;  /* [N1+N2] 2I per nucleus, 1..RP_MAX_TWO_I */
  const double *a_mT;    /* [N1+N2] isotropic hyperfine constants a_ik/gamma in mT (Eq. 1) */
  double J_mT;           /* exchange J/gamma in mT: term 2 J S1.S2 of Eq. 1 */
  double kS, kT;         /* singlet and triplet recombination rate constants, 1/us, >= 0 (Eq. 2) */
  double T_us;           /* upper limit of the yield integral (Eq. 20, 22 taken on [0, T]), > 0 */
  double gamma;          /* electron gyromagnetic ratio in rad/us/mT; 0 selects 176.085963023 */
} rp_system;

/* Propagation options.  Zero-initialised options select the defaults. */
typedef struct rp_opts {
  int32_t precision;        /* 64: complex FP64 wavepackets; 32: complex FP32 wavepackets with FP64
                               coefficients, bounds and yield accumulation.  0 selects 64. */
  int32_t init_mode;        /* 0: angles hold (cos theta, phi) per nucleus: coherent states (Eq. 15);
                               1: angles[..][0] holds the digit n = I - m per nucleus: the basis
                               state |S, M_1, M_2> of Eq. 12 (the [..][1] entry is ignored). */
  double tol;               /* Chebyshev truncation tolerance; 0 selects 1e-14 (64) or 1e-9 (32) */
  double rdt;               /* target r*dt of one Chebyshev step (r = spectral half-width); 0 = 100 */
  double r_scale;           /* multiplies the spectral half-width bound; 0 selects 1.  Values below 1
                               under-estimate the spectrum and exist to test RP_ENOTCONV. */
  int64_t workspace_bytes;  /* cap on the device memory of the wavepacket chunks of a call (the call's
                               coefficient tables come on top); 0 selects half of free memory */
  int32_t flags;            /* bit mask of RP_FLAG_* */
  int32_t krylov_dim;       /* Krylov dimension m of the short-iterative Arnoldi propagator
                               (RP_FLAG_ARNOLDI); 0 selects 16, otherwise 2..32 */
  double max_growth;        /* bound on the growth of the Chebyshev vectors over one step, worst case
                               over the dissipative strip of the spectrum; steps are shortened until
                               it holds (it limits the rounding error of the series).  0 selects
                               1e10 (64) or 1e6 (32); otherwise >= 2. */
  int64_t ps_t_len;         /* time points per wavepacket in rp_propagate's ps_t (required, >= 1,
                               when ps_t is not NULL; ignored otherwise) */
} rp_opts;

/* opts->flags: record HIP events around the Chebyshev-term launches of every step
   and keep the totals for rp_profile_last (adds a few event records per step). */
#define RP_FLAG_PROFILE 1
/* opts->flags: use the tiled kernels for every system.  Without it, systems with at most
   1024 (complex FP32) or 512 (FP64) nuclear states run in the LDS-resident kernel: one
   workgroup per wavepacket for the whole propagation, every such job of the call in one
   launch per workgroup size.  Profiled calls always use the tiled kernels. */
#define RP_FLAG_TILED 2
/* opts->flags: workgroup order of the tiled kernels.  By default each XCD takes a contiguous
   eighth of a launch's tiles (whole wavepackets when there are eight or more, so their partner
   tiles stay in one XCD's L2) while a wavepacket (4Z complex values) is at most 32 MB, and
   larger ones are spread round-robin over all XCDs; these flags force one or the other (for
   tuning). */
#define RP_FLAG_XCD_LOCAL 4
#define RP_FLAG_XCD_SPREAD 8
/* opts->flags: launch the tiled kernels directly instead of replaying one captured HIP graph
   per step (graphs are captured per number of active wavepackets and buffer parity, on a
   stream of the library's own when the caller passes the legacy default stream). */
#define RP_FLAG_NO_GRAPH 16
/* opts->flags: propagate with the short-iterative Arnoldi method the paper names (Sec. III)
   instead of the Chebyshev series: per step an m-dimensional Krylov space of A = H + i beta P_S
   (Eq. 1-4 without the scalar decay k_T/2), the step length from the Arnoldi error estimate
   (local error <= opts->tol, default 1e-13 for 64 and 1e-8 for 32), the in-step yield from
   the projected singlet Gram matrix by Van Loan's block exponential.  Same outputs and units;
   for comparison with the default propagator (every job of a call does the same launches,
   each with its own step length; the small Krylov algebra runs on the host in FP64). */
#define RP_FLAG_ARNOLDI 32
/* opts->flags: run the complex-FP32 Chebyshev terms with one nuclear index per thread (the
   256-index tile kernel, 8-byte accesses) instead of two per thread with 16-byte accesses.
   Same sums in the same order; for comparison. */
#define RP_FLAG_TERM_SCALAR 64
/* opts->flags: internal nuclear axis order with the higher spins on the fastest axes (and the
   mixed-radix term kernel) instead of the spin-1/2 nuclei first (the 256-index tile kernels).
   Same yields up to rounding; a candidate of the autotuner for systems that mix spins. */
#define RP_FLAG_AXES_HIGH_FIRST 128

/*
 * rp_sample -- directions of the nuclear coherent states (Eq. 18: uniform on
 * each sphere, measure dOmega / 4 pi), or basis-state digits.
 *
 *   s            system (only N1+N2 and two_I are read)
 *   seed, stream_id  Philox4x64-10 key (seed, stream_id); stream ids separate
 *                uses (0 evaluation, 1 training, 2 quadrature, 3 spare)
 *   first_sample global index of the first sample (counter word 0)
 *   M            number of samples, >= 0
 *   basis_mode   0: coherent-state directions (cos theta, phi), with
 *                   cos theta = 2 u1 - 1, phi = 2 pi u2, u = (floor(w/2^12) + 1/2) 2^-52
 *                   from words 0 and 1 of Philox(counter = (sample, nucleus, 0, 0));
 *                1: random basis states, digit n = floor(u1 (2I+1)) (Sec. V, last
 *                   paragraph: sampling of J_z eigenstates);
 *                2: deterministic enumeration, sample s -> digits of s in the mixed
 *                   radix of the nuclei (first nucleus fastest), for the Eq. 14 sum;
 *                3, 4, 5: coherent-state directions in sign-flip designs, a variance
 *                   reduction of the Eq. 18 mean (the measure of Eq. 17 is invariant under
 *                   n -> -n).  The global sample index q = first_sample + s lies in group
 *                   q / R, row q % R, with R = rp_design_size(N1+N2, basis_mode).  The
 *                   group draws directions as mode 0 does for sample index q / R; row r
 *                   maps n_k -> -n_k (cos theta -> -cos theta, phi -> phi + pi, reduced
 *                   below 2 pi) where its sign is -1.
 *                   Mode 3: antithetic pair, R = 2, row 1 flips every nucleus.
 *                   Mode 4: fold-over of the Sylvester-Hadamard matrix of order n (the
 *                   smallest power of two >= N1+N2), R = 2n; sign of nucleus k in row r is
 *                   (-1)^popcount((r mod n) & k), negated for r >= n: an orthogonal array
 *                   of strength 3.
 *                   Mode 5: columns 1.. of the Sylvester-Hadamard matrix of order R, the
 *                   smallest power of two > N1+N2; sign (-1)^popcount(r & (k+1)): an
 *                   orthogonal array of strength 2.
 *                   Each sample is marginally uniform, so each group's mean is unbiased and
 *                   the groups are independent: take the error from group means
 *                   (rp_group_mean, then rp_yield), with first_sample and M multiples of
 *                   R.  Use init_mode 0 in rp_propagate.
 *   angles       device, [M][N1+N2][2] doubles, written.
 */
int rp_sample(const rp_system *s, uint64_t seed, uint32_t stream_id, uint64_t first_sample,
              int64_t M, int32_t basis_mode, double *angles, void *hip_stream);

/*
 * rp_design_size -- samples per group R of rp_sample's basis_mode for n_nuclei nuclei: 1 for
 * modes 0-2, 2 for mode 3, 2n for mode 4 (n the smallest power of two >= n_nuclei), the
 * smallest power of two > n_nuclei for mode 5.  Host only; returns RP_EINVAL (negative) for
 * a mode outside 0..5 or n_nuclei outside 0..RP_MAX_NUCLEI.
 */
int64_t rp_design_size(int32_t n_nuclei, int32_t basis_mode);

/*
 * rp_propagate -- single-wavepacket singlet yields phi_S (Eq. 22 on [0, T]) for
 * every system, field and sample.
 *
 *   sys        [n_sys] systems
 *   B_mT       host, [n_sys][nB] field strengths in mT
 *   angles     device, the concatenation over systems of [M][N_i][2] arrays as
 *              written by rp_sample (interpretation set by opts->init_mode)
 *   M          samples per system
 *   opts       options (NULL = defaults)
 *   phi        device, [n_sys][nB][M] doubles, written
 *   ps_t       device, [n_sys][nB][M][opts->ps_t_len] doubles, or NULL: the singlet
 *              population <psi(t)|P_S|psi(t)> (Eq. 3 and Eq. 20 without the factor k_S; it
 *              includes the loss of norm by recombination) at the start of every step,
 *              t_j = j dt for j < min(ps_t_len, n_steps), with dt and n_steps of that system
 *              and field as rp_plan_field reports them (info[3], info[4]); NaN for j >=
 *              n_steps.  Written by the tiled kernels (small systems then run tiled too);
 *              RP_ENOTIMPL with RP_FLAG_ARNOLDI (adaptive steps have no common time grid).
 *
 * Each wavepacket is propagated by a Chebyshev expansion of exp(-iGt),
 * G = H - iK, in steps of length dt; the time integral of P_S within each step
 * is exact up to the truncation tolerance (Gauss-Legendre integrals of products
 * of Bessel functions, factored by pivoted Cholesky).  With RP_FLAG_ARNOLDI the
 * short-iterative Arnoldi propagator is used instead (see that flag).
 *
 * Several systems in one call: systems with at most 1024 (complex FP32) or 512 (FP64)
 * nuclear states run in the LDS-resident kernel; the others share one job queue per term
 * kernel, so that wavepackets of unequal Z are propagated by the same launches.
 *
 * Workspace: one block of device memory per call, taken on hip_stream with hipMallocAsync
 * and returned with hipFreeAsync (stream-ordered; hipMalloc / hipFree where that is not
 * available): the call's tables plus the largest chunk of wavepackets (three vectors of 4Z
 * complex numbers per job plus the singlet amplitudes of one step, N_terms x Z per job),
 * with chunks cut so that the chunk buffers stay within opts->workspace_bytes, else the
 * whole block within half of the free memory.
 */
int rp_propagate(const rp_system *sys, int32_t n_sys, const double *B_mT, int32_t nB,
                 const double *angles, int64_t M, const rp_opts *opts, double *phi, double *ps_t,
                 void *hip_stream);

/*
 * rp_propagate_static -- rp_propagate without any device allocation, for callers that cannot
 * allocate device memory (code near graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, outputs and errors as rp_propagate; the caller still passes the
 * inputs and outputs.
 *
 * Workspace: a static device area of RP_STATIC_SCRATCH_MB MiB that the library holds on every
 * GPU it runs on (its own copy per GPU) until the process ends, instead of a per-call
 * allocation.  Calls whose tables plus one wavepacket's buffers (three vectors of 4Z complex
 * numbers and N_terms x Z singlet amplitudes) exceed it return RP_ENOMEM with the sizes in
 * rp_last_error(); larger calls are cut into chunks that fit.  opts->workspace_bytes must be
 * 0; RP_FLAG_ARNOLDI and RP_FLAG_PROFILE return RP_ENOTIMPL.  Kernels are launched directly
 * (no internal graph capture; every buffer clear is a kernel, not a memset), and the call
 * waits for its work before returning, as rp_propagate does.
 *
 * Every call on a GPU shares that GPU's area and leaves its last contents there: calls that
 * overlap on one GPU (several host threads, or several streams without ordering between the
 * calls) race and must be serialised by the caller.
 */
#define RP_STATIC_SCRATCH_MB 256
int rp_propagate_static(const rp_system *sys, int32_t n_sys, const double *B_mT, int32_t nB,
                        const double *angles, int64_t M, const rp_opts *opts, double *phi, double *ps_t,
                        void *hip_stream);

/*
 * rp_yield -- per-field Monte Carlo mean and standard error (Eq. 18, Eq. 23:
 * eps = s / sqrt(M), s with the 1/(M-1) normalisation).
 *
 *   phi       device, [nB][M] single-wavepacket yields
 *   cv_g      device [nB][M] control-variate values g, or NULL for the plain mean
 *   cv_mu     device [nB] known means of g (ignored when cv_g is NULL)
 *   cv_beta   device [nB] coefficients (ignored when cv_g is NULL); the estimate is
 *             mean(phi - beta (g - mu)), unbiased when E[mu] = E[g] and beta is fixed
 *             independently of the M samples
 *   cv_mu_err device [nB] standard error of mu (mu taken from independent samples), or NULL
 *             for 0; (beta cv_mu_err)^2 is added to stderr^2
 *   mean, stderr_  device [nB] outputs
 */
int rp_yield(const double *phi, int32_t nB, int64_t M, const double *cv_g, const double *cv_mu,
             const double *cv_beta, const double *cv_mu_err, double *mean, double *stderr_,
             void *hip_stream);

/*
 * rp_group_mean -- means of consecutive groups of samples: out[b][j] = (1/group)
 * sum_{i < group} phi[b][j group + i], summed in order in FP64.  For the sign-flip designs of
 * rp_sample (modes 3-5) each group mean is one independent unbiased estimate of the Eq. 18
 * trace; rp_yield over the M / group means gives the design estimate and its standard error
 * (Eq. 23 with the groups as samples).
 *
 *   phi    device, [nB][M] doubles
 *   group  samples per group, >= 1 and dividing M (else RP_EINVAL)
 *   out    device, [nB][M / group] doubles, written
 */
int rp_group_mean(const double *phi, int32_t nB, int64_t M, int64_t group, double *out, void *hip_stream);

/*
 * Learned control variate (for the Monte Carlo mean of Eq. 18).  A network g(Omega, B)
 * with features x = (n(Omega_1), ..., n(Omega_N), log(B/mT + 0.05)) (unit vectors of Eq. 16),
 * `depth` hidden layers of `width` units with exact-erf GELU, and a scalar output, is trained
 * by mean-squared error on yields phi_S produced by rp_propagate.  Hidden-layer products run
 * on MFMA with BF16 inputs and FP32 accumulation; parameters, Adam moments and gradients are
 * FP32.  For callers who cannot guess the padded input width: n_in_pad = 16 * ceil(n_in / 16).
 *
 * Packed parameter layout (FP32, device): for each hidden layer l, W_l [fan_in][width]
 * (fan_in = n_in_pad for l = 0, else width) then b_l [width]; then the output weights
 * w [width] and the output bias (1 value).
 *
 * rp_mlp_param_count     number of packed parameters (-1 for a bad shape: width must be a
 *                        positive multiple of 16, 1 <= depth <= 8).
 * rp_mlp_workspace_floats  FP32 workspace needed by forward/train calls on `rows` rows.
 * rp_mlp_features        x[row][0 .. n_in_pad) (device), nB*M rows, device fields B_mT [nB]:
 *                        layout 0: [M][N][2] angles shared by all fields, row = b*M + s;
 *                        layout 1: the same angles, row = s*nB + b (batches mix fields);
 *                        layout 2: [nB*M][N][2] angles, one per row, row r has field r % nB.
 *                        rot_seed != 0 advances every azimuth of row r by 2 pi u_r, u_r from
 *                        SplitMix64(rot_seed + (r+1) * 0x9E3779B97F4A7C15) (top 53 bits +
 *                        1/2, times 2^-53): a common rotation of the nuclear directions about
 *                        the field, under which the yield is exactly invariant (training-data
 *                        augmentation; 0 for inference).
 * rp_mlp_forward         y[rows] = g(x) (device).
 * rp_mlp_train_step      one Adam step (beta1 0.9, beta2 0.999, eps 1e-8; step >= 1 is the
 *                        Adam time step) on the batch (x, target); optional device outputs:
 *                        grad_out [param_count] (the gradient of the mean squared error) and
 *                        sq_err [rows] (squared errors before the update).  lr = 0 computes
 *                        gradients without updating.
 */
/*
 * rp_mlp_standardize    training targets standardised per field: phi (device, doubles) has
 *                       rows q = s * nB + b (s < n_rows, field b); with the mean and standard
 *                       deviation (1/n normalisation; 1 where it is 0) of field b over its first
 *                       n_fit rows, target[q] = (phi[q] - mean_b) / std_b (device floats).
 * rp_mlp_loss           mean squared error of g(x) against target over `rows` rows, into the
 *                       device double *mse (the validation loss of early stopping).
 */
int rp_mlp_standardize(const double *phi, int32_t nB, int64_t n_rows, int64_t n_fit, float *target,
                       void *hip_stream);
int rp_mlp_loss(int32_t n_in, int32_t width, int32_t depth, const float *params, const float *x,
                const float *target, int64_t rows, double *mse, float *workspace, void *hip_stream);
int64_t rp_mlp_param_count(int32_t n_in, int32_t width, int32_t depth);
int64_t rp_mlp_workspace_floats(int32_t n_in, int32_t width, int32_t depth, int64_t rows);
int rp_mlp_features(const double *angles, int64_t M, int32_t N, const double *B_mT, int32_t nB,
                    int32_t n_in_pad, int32_t layout, uint64_t rot_seed, float *x, void *hip_stream);
int rp_mlp_forward(int32_t n_in, int32_t width, int32_t depth, const float *params, const float *x,
                   int64_t rows, float *y, float *workspace, void *hip_stream);
int rp_mlp_train_step(int32_t n_in, int32_t width, int32_t depth, float *params, float *adam_m,
                      float *adam_v, int64_t step, const float *x, const float *target, int64_t rows,
                      float lr, float *grad_out, float *sq_err, float *workspace, void *hip_stream);

/*
 * rp_profile_last -- timing of the most recent rp_propagate call on the calling
 * thread that had RP_FLAG_PROFILE set.  out (host, n <= 8 doubles):
 *   [0] milliseconds spent in Chebyshev-term kernels (events on the call's stream)
 *   [1] number of Chebyshev-term kernel launches
 *   [2] wavepacket elements processed by them (sum over launches of jobs * 4Z)
 *   [3] algorithmic bytes per element and term, averaged over the launches: a term
 *       reads phi_n and phi_{n-1} and writes phi_{n+1} and the singlet amplitude
 *       (26 bytes per element for complex FP32); every third term also reads and
 *       writes the step accumulator (+16); the first term of a step reads phi_0 and
 *       writes phi_1, the accumulator and two amplitudes (28).  Doubled for FP64.
 *   [4] milliseconds in the in-step quadrature kernels, [5] their launches
 *   [6] milliseconds of the whole call, [7] Chebyshev terms per step (padded maximum)
 * With RP_FLAG_ARNOLDI only [5] (Arnoldi steps, summed over jobs) and [7] (applications of
 * H + i beta P_S, summed over jobs) are filled; the others are 0.
 * Returns the number of values written.
 */
int rp_profile_last(double *out, int32_t n);

/*
 * rp_combine -- per field, the inverse-variance weighted mean of two independent unbiased
 * estimates of the same yield (Eq. 18 applied to two disjoint sample sets, e.g. the plain
 * mean of the control variate's training yields and the control-variate estimate on the
 * evaluation samples):  mean = (ma/ea^2 + mb/eb^2) / (1/ea^2 + 1/eb^2),  err = (1/ea^2 +
 * 1/eb^2)^(-1/2); an estimate with zero error is taken as it is.  All arrays device [nB].
 * The weights use estimated errors, so the combination carries a bias of relative order 1/M
 * against the errors themselves.
 */
int rp_combine(const double *mean_a, const double *err_a, const double *mean_b, const double *err_b, int32_t nB,
               double *mean, double *err, void *hip_stream);

/*
 * rp_cv_beta -- per-field control-variate coefficient beta_b = Cov(phi, g) / Var(g) over the
 * M samples (the variance-minimising coefficient), from device phi, g [nB][M] to device
 * beta [nB] (0 where Var(g) = 0).  Take it from samples independent of the evaluation set.
 */
int rp_cv_beta(const double *phi, const double *g, int32_t nB, int64_t M, double *beta, void *hip_stream);

/*
 * rp_probe_stream -- measurement helper: the practical HBM ceilings the term kernel is quoted
 * against.  Times `reps` launches (after one warm-up) of plain streaming kernels over `bytes`
 * bytes (a multiple of 16) with 16-byte vector accesses, on hip_stream, and waits for them;
 * three variants (one or four vectors per thread, plain or non-temporal) are timed and the
 * fastest counts.  kind 0: c = a (reads and writes `bytes` each); 1: c = a + b (two reads, one write);
 * 2: reads a only; 3: writes c only.  a, b, c: device buffers of `bytes` bytes (b only for
 * kind 1, a not for kind 3).  *ms_per_launch (host) receives the average launch time.
 */
int rp_probe_stream(int32_t kind, const void *a, const void *b, void *c, int64_t bytes, int32_t reps,
                    double *ms_per_launch, void *hip_stream);

/* Static text for a return code. */
const char *rp_strerror(int code);

/* Message for the most recent failure on the calling thread ("" if none). */
const char *rp_last_error(void);

/*
 * Host-only planning helpers (no device work; used to test the propagator's
 * coefficients on a machine without a GPU).
 *
 * rp_bessel_j: J_0(x) .. J_nmax(x) for x >= 0 by Miller's backward recurrence
 *   normalised with J_0 + 2 sum_k J_2k = 1.  out: host [nmax+1].
 *
 * rp_plan_field: the Chebyshev step plan for one system at one field.
 *   info (host, 8 doubles): r, c_re, c_im, dt, n_steps, n_terms (N+1), rank R, x = r dt
 *   coef (host or NULL, 2*n_terms doubles): complex a_n of one step, interleaved re/im
 *   ell  (host or NULL, n_terms*R doubles): real factor of the in-step quadrature,
 *        row n, column r, including the (2 - delta_n0) and 1/sqrt(2) factors
 */
int rp_bessel_j(double x, int32_t nmax, double *out);
int rp_plan_field(const rp_system *s, double B_mT, const rp_opts *opts, double *info, double *coef,
                  double *ell);

#ifdef __cplusplus
}
#endif

#endif /* RP_H */
