/*
 * rteom.h -- C ABI of the MI355X RT-EOM-CCSD hot path (arXiv 2301.04249).
 *
 * The library propagates the complex CCSD amplitudes of a core-ionised
 * (N-1)-electron reference in time and accumulates the cumulant C(t):
 *
 *   -i dt_x/dtau = <Phi_x|(H_N e^{T1+T2})_C|Phi>          (Eqs. dt1eom, dt2eom)
 *   T(tau+dt) = T(tau) + (i dt/2)[R(T(tau)) + R(T(tau+dt))] (Eq. trapzrule)
 *   C(tau) = i int_0^tau <Phi|(H_N e^{T})_C|Phi> dtau'      (Eq. cum_gf3)
 *
 * with the two-electron integrals Cholesky factorised,
 * (pq|rs) = sum_Q L^Q_pq L^Q_rs (Sec. 2.3), spin-explicit (alpha-alpha,
 * alpha-beta, beta-beta) amplitude blocks, and the (N-1) Fock matrix
 * f_pq = eps_p delta_pq - <pc||qc> (Sec. 2.1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns rteom_status (0 = RTEOM_OK).  Nothing aborts and no
 *   C++ exception crosses the ABI; rteom_last_error() gives a message.
 * - Pointers named "host" are CPU memory owned by the caller; they are read or
 *   written during the call only.  Device memory is either the caller's
 *   workspace (rteom_options.workspace, e.g. a torch tensor) or allocated by
 *   the library when that pointer is NULL; rteom_free releases what the
 *   library allocated and never the caller's workspace.
 * - Work is ordered on rteom_options.stream (a hipStream_t, NULL = the null
 *   stream).  Calls that return host data synchronise that stream.
 * - Orbital spaces: the N-electron determinant occupies spatial orbitals
 *   0..n_occ_a-1 (alpha) and 0..n_occ_b-1 (beta); the core spin-orbital
 *   (core_orb, core_spin) is removed to make |Phi>.  The library works in an
 *   "extended" space: O = orbitals occupied in Phi in either spin (ascending),
 *   V = orbitals virtual in Phi in either spin (ascending), n_o = |O|,
 *   n_v = |V|.  Amplitudes of a spin that does not exist (e.g. beta
 *   amplitudes with i = core) are identically zero.
 * - Host amplitude layout (rteom_set_amplitudes / get / residual): complex
 *   numbers as interleaved (re, im) doubles;
 *     t1: [2 spins][n_o][n_v]                              (alpha, beta)
 *     t2: [2 spins][P_o][P_v], then [n_o][n_o][n_v][n_v]   (aa, bb pairs; ab)
 *   with P_o = n_o (n_o - 1) / 2, P_v = n_v (n_v - 1) / 2.
 *   t1[s][i][a] = t_{i s}^{a s}.  The same-spin doubles t_{i s, j s}^{a s, b s}
 *   are antisymmetric in (i, j) and in (a, b): only i < j, a < b are stored, at
 *   pair positions p(i, j) = i (2 n_o - i - 1) / 2 + j - i - 1 and likewise
 *   p(a, b) over n_v (lexicographic pairs).  The alpha-beta block holds
 *   t_{i alpha, j beta}^{a alpha, b beta} at [i][j][a][b].  The device sets use
 *   the same order, planar (all real parts, then all imaginary parts).
 */
#ifndef RTEOM_H
#define RTEOM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rteom_ctx rteom_ctx;
typedef struct rteom_batch rteom_batch;

typedef enum {
  RTEOM_OK = 0,
  RTEOM_ERR_ARG = 1,        /* invalid argument (sizes, indices, dt, options) */
  RTEOM_ERR_OOM = 2,        /* workspace too small or device allocation failed */
  RTEOM_ERR_HIP = 3,        /* a HIP runtime call failed */
  RTEOM_ERR_NOCONV = 4,     /* fixed point not converged; the step is not committed (T, C(t) unchanged) */
  RTEOM_ERR_NONFINITE = 5,  /* NaN/Inf in the inputs, or in the amplitudes or C(t) during a step */
  RTEOM_ERR_STATE = 6       /* call not valid in the context's current state */
} rteom_status;

typedef enum {
  RTEOM_FP64 = 0,   /* contractions in float64 (MFMA f64) */
  RTEOM_FP32 = 1,   /* contractions in float32 (MFMA f32), float64 storage */
  RTEOM_BF16X3 = 2, /* bf16 hi/lo split, three MFMA products, float32 accumulation */
  RTEOM_FP16X3 = 3  /* fp16 hi/lo split of operands scaled per row by powers of two, three
                       MFMA f16 products, float32 accumulation (about float32's accuracy at
                       the 16-bit MFMA rate); products too small to convert run in float32 */
} rteom_prec;

/* Memory plan.  Every intermediate that grows like o^2 v^2 or faster is produced in
   blocks when the whole would not fit: the ring intermediates W[(m,e),(b,j)] in blocks
   of occupied columns j, expanded same-spin amplitudes in blocks of rows, and -- when
   they cannot stay resident -- the integral blocks (ae|bf), (me|bf) and their
   same-spin pair forms, rebuilt from the Cholesky vectors in slabs of virtual indices
   for every residual evaluation (Sec. 2.3).  rteom_init picks the largest blocks whose
   workspace fits rteom_options.mem_limit (and the caller's workspace); every element is
   computed by the same arithmetic under any plan. */

typedef struct {
  uint32_t struct_size;    /* must be sizeof(rteom_options) */
  int32_t prec;            /* rteom_prec of the contractions; update and C(t) stay float64 */
  int32_t fp_map;          /* 0: plain fixed point of Eq. trapzrule; 1: diagonal ("denominator") map */
  int32_t fp_fixed_iters;  /* > 0: exactly this many corrector passes per step (no convergence test);
                              1 keeps no right-hand-side amplitude set */
  int32_t fp_max_iter;     /* pass limit when tolerance driven */
  double fp_tol;           /* max |T^(k+1) - T^(k)| over all amplitudes that ends the passes */
  int32_t dC_include_fT1;  /* 1: dC/dt includes sum f_ia t_ia (Eq. cum_gf3); 0: Eq. dcdt as printed */
  int32_t graph;           /* 1: with fp_fixed_iters > 0 and a non-null stream, each time step
                              is captured once as a hipGraph and replayed; rteom_init then
                              runs one residual outside capture (GEMM tile timing with
                              tune = 1, and the converted integral planes of FP32 / BF16X3) */
  int64_t max_steps;       /* capacity of the device C(t) history (time steps) */
  void* stream;            /* hipStream_t borrowed from the caller; NULL = null stream */
  void* workspace;         /* caller-owned device memory, or NULL (library allocates) */
  size_t workspace_bytes;  /* size of workspace */
  int32_t tune;            /* 1: the first time a GEMM shape is met outside graph capture, each
                              candidate tile shape is timed on it and the fastest is kept for
                              the context (results are bit-identical for every tile shape);
                              0: tile shape from a rule (choices loaded with
                              rteom_tile_cache_load are used first either way) */
  int32_t fp_anderson;     /* 0..8: history depth m of Anderson acceleration of the
                              tolerance-driven fixed point (fp_fixed_iters = 0) and of
                              rteom_ground_state: each pass mixes the last m results
                              G(x_j) with the weights (sum 1) that minimise the norm of
                              the mixed G(x_j) - x_j; 0 = plain iteration.  Costs 2 m
                              amplitude sets of workspace. */
  size_t mem_limit;        /* bytes the memory plan may use (0 = 270 GiB: MI355X HBM less
                              room for the runtime); a caller's workspace lowers it */
  int32_t plan_slab;       /* 0: automatic plan; > 0: the integral blocks are rebuilt per
                              residual in slabs of this many virtual indices */
  int32_t plan_block;      /* 0: automatic; > 0: occupied indices per block of the ring
                              intermediates and of the expanded same-spin rows.  With either
                              set, the plan is used as given (OOM if it does not fit). */
  int32_t progress;        /* 1: a residual evaluation that runs in blocks waits for the
                              stream after each ring block and integral slab and writes one
                              line per block to stderr (elapsed seconds): long evaluations
                              report where they are */
} rteom_options;

/* Fill *opt with defaults: FP64, plain map, tolerance 1e-10, 50 passes,
   dC_include_fT1 = 1, no graph, max_steps = 100000, null stream, no workspace, tune = 1. */
void rteom_default_options(rteom_options* opt);

/* Device bytes rteom_init needs for these sizes and options (no GPU work) under the
   memory plan it would choose: three amplitude sets (two with fp_fixed_iters = 1; plus
   T_n for tolerance-driven steps and the Anderson history), the Cholesky vectors and
   resident integral blocks, and the scratch of one residual evaluation.  OOM if no plan
   fits mem_limit. */
rteom_status rteom_workspace_query(int32_t n_orb, int32_t n_occ_a, int32_t n_occ_b,
                                   int32_t n_chol, int32_t core_orb, int32_t core_spin,
                                   const rteom_options* opt, size_t* bytes);

/* Create a propagation context (Sec. 3, the time-dependent simulation of one core hole).
   fock_diag: host [n_orb], the N-electron orbital energies eps_p (Fock diagonal).
   chol:      host [n_chol][n_orb][n_orb], Cholesky vectors L^Q_pq, symmetric in (p,q).
   core_orb/core_spin: the ionised spin-orbital c (spatial index occupied in that spin,
   0 = alpha, 1 = beta); core_orb = -1 makes the N-electron determinant itself the
   reference (no ionisation, core_spin ignored: for rteom_ground_state).  Builds the
   Fock matrix of the reference and the integral blocks on the device; T(0) = 0 and
   C(0) = 0.  The caller may free the host arrays afterwards.
   Errors: ARG (sizes, indices, non-symmetric L), NONFINITE, OOM, HIP. */
rteom_status rteom_init(rteom_ctx** ctx, int32_t n_orb, int32_t n_occ_a, int32_t n_occ_b,
                        const double* fock_diag, int32_t n_chol, const double* chol,
                        int32_t core_orb, int32_t core_spin, const rteom_options* opt);

/* Advance n_steps time steps of length dt (Eq. trapzrule with fixed-point passes) and
   append C(t) for each (Eq. cum_gf3).  micro_iters_out (nullable, host [n_steps])
   receives the passes used per step.  Synchronises the stream.
   Tolerance-driven steps (fp_fixed_iters = 0) keep T_n (one more amplitude set of
   workspace): a step whose fixed point does not converge within fp_max_iter passes
   (NOCONV) or whose iterate turns NaN/Inf (NONFINITE) is not committed -- T and C(t)
   stay at the last committed step and the context remains usable (e.g. with a smaller
   dt).  Fixed-pass and graph-replayed steps check once per call, after the stream has
   drained, a device flag that the C(t) append raises when E(T) or C(t) is not finite
   (E sums every amplitude times an integral, so one NaN/Inf amplitude makes it so):
   then NONFINITE, C(t) holds the appended steps, and the context is in a failed state
   (STATE) until amplitudes are set or a checkpoint is restored. */
rteom_status rteom_step(rteom_ctx* ctx, double dt, int32_t n_steps, int32_t* micro_iters_out);

/* Copy the cumulant history to host (Eq. cum_gf3: C(tau) = i int_0^tau
   <Phi|(H_N e^T)_C|Phi> dtau', accumulated with the trapezoid weights of the time grid,
   C(0) = 0): t_out [cap] times, c_out [cap][2] (re, im) of C(t_0 = 0) ... C(t_n);
   *n_out = number written (steps taken + 1, at most cap).  cap = 0 is a length query:
   nothing is written and *n_out = steps taken + 1.  Synchronises the stream. */
rteom_status rteom_cumulant(const rteom_ctx* ctx, int64_t cap, double* t_out, double* c_out,
                            int64_t* n_out);

/* Ground-state CCSD of the reference (Sec. 2.2: the correlation energy E_N^corr of the
   N-electron ground state enters the phase of G(t), see rteom_spectral): solves
   R(T) = 0 (Eqs. dt1eom, dt2eom with the left side zero) by Jacobi iteration
   T <- T + R(T) / D (D the orbital-energy denominators), from T = 0, until the largest
   change of an amplitude is below tol, and writes E^corr = <Phi|(H_N e^T)_C|Phi>
   (Eq. cum_gf3's integrand) to host e_corr [2] = (re, im).  Meant for a context created
   with core_orb = -1; the converged amplitudes replace the context's (the C(t) history
   is untouched).  iters (nullable): Jacobi iterations used.  ARG for tol <= 0 or
   max_iter < 1; NOCONV / NONFINITE leave the context in a failed state. */
rteom_status rteom_ground_state(rteom_ctx* ctx, double tol, int32_t max_iter, double* e_corr, int32_t* iters);

/* Checkpoint and restart of a propagation (Sec. 3: runs of hundreds of atomic time units
   need restarts).  The image holds the amplitudes T(t_n), the C(t) and E(t) histories and
   the time grid t_0..t_n, behind a header (magic, version, n_orb, n_occ_a, n_occ_b,
   n_chol, core_orb, core_spin, steps); integrals are not stored, the caller re-creates
   the context from its inputs.  rteom_checkpoint: buf NULL -> *bytes = image size, OK;
   cap < size -> *bytes = size, ARG; else the image is written to host buf.  STATE if the
   context is in a failed state.  Synchronises the stream. */
rteom_status rteom_checkpoint(rteom_ctx* ctx, void* buf, size_t cap, size_t* bytes);

/* Restore an image written by rteom_checkpoint (host buf of len bytes) into a context
   created with the same sizes and core orbital: amplitudes, histories and step count
   are replaced and a failed state is cleared; options (precision, map, graph) are the
   context's own.  ARG for a truncated or foreign image, mismatched sizes, or more steps
   than the context's max_steps. */
rteom_status rteom_restore(rteom_ctx* ctx, const void* buf, size_t len);

/* Spectral function of the core hole from the device C(t) history (Sec. 2.2: the
   cumulant form of the core Green's function, Eqs. cum_gf and cum_gf2):
     G(t_k) = -i exp(-i (eps_c + e_corr) t_k) exp(C(t_k)),
     A(w)   = -(1/pi) Im sum_k w_k exp(i w t_k - eta t_k) G(t_k),
   with eps_c the Fock-diagonal entry of the ionised orbital given to rteom_init,
   e_corr the N-electron correlation energy (a constant shift; 0 if unknown), w_k
   the trapezoid weights of the time grid and eta >= 0 a damping (Lorentzian
   broadening).  omega: host [n_w] frequencies (Eh), ascending and uniformly
   spaced for the peak refinement; a_out: host [n_w] A(omega).  qp_out (nullable):
   host [2] = (position of the largest A, refined by the parabola through the
   grid maximum and its two neighbours; A at the grid maximum).  Computed on the
   device (temporary device memory of (3 n + 2 n_w + 2) doubles, n = steps + 1);
   synchronises the stream.  ARG for NULL omega/a_out, n_w < 1, non-finite
   input, eta < 0 or a context without a core hole; OOM if the temporary cannot be
   allocated. */
rteom_status rteom_spectral(rteom_ctx* ctx, double e_corr, double eta, int64_t n_w, const double* omega,
                            double* a_out, double* qp_out);

/* Quasi-particle peak and satellites of the spectral function (Sec. 3: the main line and its
   satellites; Eqs. cum_gf, cum_gf2): A(omega) as rteom_spectral computes it (written to
   a_out [n_w] if not NULL), then its local maxima (A_j > A_{j-1} and A_j >= A_{j+1},
   0 < j < n_w - 1), the largest first (first index on ties), at most max_peaks (1..64):
   peaks_out [max_peaks][2] = (position refined by the parabola through the maximum and
   its two neighbours, A at the grid maximum); *n_peaks = number found.  The first entry
   is the QP peak; the others are satellites (and, with a coarse grid or short
   propagation, ripples of the finite time window).  Temporary device memory of
   3 (steps + 1) + 2 n_w + 2 max_peaks + 3 doubles; synchronises the stream.  ARG for bad
   sizes or a context without a core hole; OOM if the temporary cannot be allocated. */
rteom_status rteom_spectral_peaks(rteom_ctx* ctx, double e_corr, double eta, int64_t n_w, const double* omega,
                                  double* a_out, int32_t max_peaks, double* peaks_out, int32_t* n_peaks);

/* rteom_spectral for callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the same computation,
   arguments and results, with its temporary in a fixed device array of 4194304 doubles
   (32 MiB) that the library holds on each GPU it runs on until the process ends, instead
   of a device allocation per call.  Requires 3 (steps taken + 1) + 2 n_w + 2 <= 4194304:
   ARG (with a message) beyond that, before any device work.  Calls on one GPU share the
   array: calls that overlap (other threads or streams) race.  Each call writes every
   element it reads, so the array's previous contents do not matter.  STATE if the array's
   address could not be obtained.  Synchronises the stream. */
rteom_status rteom_spectral_noalloc(rteom_ctx* ctx, double e_corr, double eta, int64_t n_w, const double* omega,
                                    double* a_out, double* qp_out);

/* Extended-space sizes and orbital lists: occ_list [n_o], vir_list [n_v] (nullable). */
rteom_status rteom_dims(const rteom_ctx* ctx, int32_t* n_o, int32_t* n_v, int32_t* occ_list,
                        int32_t* vir_list);

/* Replace the current amplitudes (host layout above).  Entries of non-existent spin
   amplitudes are ignored (set to zero).  t1 = t2 = NULL: the amplitudes have been
   written in place into the device set that rteom_device_sets returns; they are taken
   as they are (masked like host input).  Either way E(T_n) is recomputed and a failed
   state is cleared.  Test and benchmark hook. */
rteom_status rteom_set_amplitudes(rteom_ctx* ctx, const double* t1, const double* t2);

/* Device addresses of the current amplitude set (x) and of the residual set (r, written by
   rteom_residual), each *doubles doubles in the device layout (planar: the real parts of
   t1, same-spin pairs, alpha-beta block, then the imaginary parts in the same order).
   They lie in the context's workspace and stay valid until rteom_free.  For callers that
   cannot afford host copies at large sizes: write x in place, then call
   rteom_set_amplitudes(ctx, NULL, NULL); read r after rteom_residual(ctx, NULL, NULL).
   Work on them must be ordered with the context's stream.  Test and benchmark hook. */
rteom_status rteom_device_sets(const rteom_ctx* ctx, void** x, void** r, int64_t* doubles);

/* Copy the current amplitudes to host (layout above). */
rteom_status rteom_get_amplitudes(const rteom_ctx* ctx, double* t1, double* t2);

/* One residual evaluation R(T) = <Phi_x|e^{-T} H_N e^{T}|Phi> at the current amplitudes
   (Eqs. dt1eom, dt2eom).  r1_out/r2_out: host, amplitude layout; either may be NULL
   (the residual is still computed, e.g. for timing). */
rteom_status rteom_residual(rteom_ctx* ctx, double* r1_out, double* r2_out);

/* <Phi|(H_N e^T)_C|Phi> at the current amplitudes (Eq. cum_gf3), e_out = (re, im). */
rteom_status rteom_energy(rteom_ctx* ctx, double* e_out);

/* Floating-point operations of one residual evaluation in this implementation's
   formulation, over existing spin-orbitals only (real flops: 2 per real MAC, 4 per
   complex x real, 8 per complex x complex even where the kernels form a complex product
   from three real ones; same-spin doubles over their unique pairs; the integral slabs
   rebuilt per residual included).  Known from rteom_init on (the plan fixes it). */
rteom_status rteom_residual_flops(const rteom_ctx* ctx, double* flops);

/* The memory plan rteom_init chose (all outputs nullable): resident = 1 if the integral
   blocks are built once, else e_slab = virtual indices per rebuilt slab; ring_cols =
   occupied columns per block of the ring intermediates; rows = rows per block of
   expanded same-spin amplitudes; exec_flops = the flops the kernels execute per
   residual (as rteom_residual_flops, but including the extended space's padding);
   workspace_bytes = the workspace in use. */
rteom_status rteom_plan_info(const rteom_ctx* ctx, int32_t* resident, int64_t* e_slab, int64_t* ring_cols,
                             int64_t* rows, double* exec_flops, size_t* workspace_bytes);

/* Device timing by phase of the hot path: 0 particle-ladder GEMM, 1 o^3 v^3 ring / W / Z
   GEMMs, 2 other GEMMs, 3 tensor moves, 4 trapezoid update, 5 energy and C(t), 6 integral
   slabs rebuilt from the Cholesky vectors (non-resident plans).  HIP events
   are recorded around every operation of the phases whose bit is set in phase_mask, on the
   context's stream; 0 switches timing off.  For benchmarking and profiling. */
rteom_status rteom_profile(rteom_ctx* ctx, uint32_t phase_mask);

/* Statistics of one phase since the previous query of that phase: *ms device time of its
   operations (0 unless profiled), *ops operations timed, *flops the phase's flops in one
   residual evaluation (same convention as rteom_residual_flops).  Synchronises the stream. */
rteom_status rteom_phase_stats(rteom_ctx* ctx, int32_t phase, double* ms, double* flops,
                               int64_t* ops);

/* Persisted tile choices.  A context created with tune = 1 times the tile shapes of every
   new GEMM signature once and keeps the fastest; rteom_tile_cache_save writes those
   choices to a text file (a header "rteom-tiles 1 <gfx target>", then one line per
   signature: precision (+8 for converted operands), M, N, K, batch, A complex, B complex,
   A k-contiguous, B k-contiguous, split-K factor, tile shape).  rteom_tile_cache_load adds
   a file's choices to a context (later ones replace earlier ones for a signature); they
   are used before timing or the rule, with tune = 0 as well.  Tile shapes change the work
   assignment only, never the arithmetic.  Errors: ARG for a NULL argument, a file that
   cannot be opened or is malformed, another device target, or a tile shape that is not
   built for its signature (nothing is loaded then).  The file is the caller's. */
rteom_status rteom_tile_cache_save(rteom_ctx* ctx, const char* path);
rteom_status rteom_tile_cache_load(rteom_ctx* ctx, const char* path);

/* Batch of independent core-hole propagations (Sec. 3: the propagations of different core
   holes are independent of each other, so they may run at the same time).  Every context
   must be in graph mode with fixed passes, on its own stream; the batch borrows them (they
   must outlive it).  rteom_batch_step advances all of them by n_steps of dt: per step, every
   context's captured time step is replayed on that context's stream, all members before any
   wait, so that members run side by side on the device's hardware queues.  Synchronises
   every member's stream on return; then checks every
   member's non-finite flag (as rteom_step does) and returns NONFINITE naming the first
   member whose E(T) or C(t) turned NaN/Inf (that member enters its failed state). */
rteom_status rteom_batch_create(rteom_batch** batch, int32_t n, rteom_ctx* const* ctxs);
rteom_status rteom_batch_step(rteom_batch* batch, double dt, int32_t n_steps);
rteom_status rteom_batch_free(rteom_batch* batch);   /* NULL-safe; leaves the contexts */

/* Release the context (NULL-safe). */
rteom_status rteom_free(rteom_ctx* ctx);

/* Last error message of this context (or of the last failed rteom_init when ctx is NULL). */
const char* rteom_last_error(const rteom_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* RTEOM_H */
