/*
 * pst.h -- C ABI of the pst library: Fourier pseudospectral time stepping
 * on AMD Instinct MI355X (gfx950), after Cloutier, Muite & Rigge,
 * "Performance of FORTRAN and C GPU extensions for a benchmark suite of
 * Fourier pseudospectral algorithms" (arXiv 1206.3215).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Fields are device pointers to row-major [batch][ny][nx] arrays (x is
 *    the fast axis).  Complex fields are interleaved (re, im) pairs of the
 *    plan's precision: float for PST_FP32, double for PST_FP64 (the memory
 *    layout of torch.complex64 / complex128).  Half spectra of real fields
 *    are [batch][ny][nx/2+1] complex (numpy.fft.rfft2 layout).
 *  - The grid of a domain d is x_j = d.x0 + j*d.lx/nx, y_i = d.y0 +
 *    i*d.ly/ny (periodic, right end point excluded); wavenumbers are
 *    2*pi*m/L with m in {0..n/2-1, -n/2..-1}.
 *  - Forward transforms are unnormalised with kernel exp(-i k.x); inverse
 *    transforms carry the factor 1/(nx*ny).
 *  - The caller owns every field buffer (for example torch tensors): it
 *    must be contiguous, on the plan's device, 256-byte aligned and of the
 *    plan's precision.  The library never frees caller memory.  A plan owns
 *    its tables (twiddles, propagators) and, unless pst_set_workspace gave
 *    it caller memory, its workspace.
 *  - Calls are asynchronous and ordered on the plan's HIP stream, except
 *    where a function says it synchronises.  Argument errors are detected on
 *    the host before anything is launched and return PST_ERR_INVALID or
 *    PST_ERR_UNSUPPORTED with a message in pst_last_error().  Conditions
 *    found on the device (a non-finite conserved quantity, a field that
 *    nls_step, sg_step or ns_step left non-finite, a fixed-point iteration
 *    that did not converge) are latched in a device status word read by
 *    pst_sync_status().
 *  - Plans are not thread safe; use one plan per stream.  No C++ exception
 *    crosses this interface.
 *  - Supported sizes: nx, ny powers of two in [4, 8192]; batch >= 1.
 */
#ifndef PST_H_
#define PST_H_

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PST_OK = 0,
  PST_ERR_INVALID = 1,       /* bad argument (null pointer, size, dt <= 0, ...) */
  PST_ERR_UNSUPPORTED = 2,   /* valid request this library does not implement */
  PST_ERR_OOM = 3,           /* device allocation failed */
  PST_ERR_DEVICE = 4,        /* a HIP runtime call failed */
  PST_ERR_NOT_CONVERGED = 5, /* Navier-Stokes fixed point hit max_iter */
  PST_ERR_NONFINITE = 6      /* a reduction or a solver's result met Inf/NaN */
} pst_status;

typedef enum { PST_FP32 = 0, PST_FP64 = 1 } pst_prec;
typedef enum { PST_C2C = 0, PST_R2C = 1 } pst_kind;
typedef enum { PST_NLS = 0, PST_SG = 1, PST_NS = 2 } pst_eq;

typedef struct pst_plan_s* pst_plan;

typedef struct {
  double lx, ly; /* periods */
  double x0, y0; /* coordinates of grid point (0, 0) */
} pst_domain;

/* i psi_t + psi_xx + psi_yy = g |psi|^2 psi (eq. nls prints g = +1). */
typedef struct {
  pst_domain d;
  double dt, g;
} pst_nls_params;

/* u_tt - Delta u = -sin u (eq. sg). */
typedef struct {
  pst_domain d;
  double dt;
} pst_sg_params;

/* omega_t + psi_y omega_x - psi_x omega_y = nu Delta omega, Delta psi = -omega. */
typedef struct {
  pst_domain d;
  double dt, nu;
  double tol;      /* stop when integral (omega^{k} - omega^{k+1})^2 < tol */
  int max_iter;    /* cap on fixed-point iterations per step (>= 1) */
  int fixed_iters; /* > 0: run exactly this many iterations, ignore tol */
} pst_ns_params;

/* ----------------------------------------------------------------- plans -- */

/* Create a plan for batch independent nx-by-ny fields of kind C2C (complex
 * fields: the FFT and the NLS solver) or R2C (real fields: the real FFT, the
 * sine-Gordon and Navier-Stokes solvers), on HIP stream hip_stream (NULL =
 * the null stream).  Builds the twiddle tables in double precision and
 * rounds them once to prec.  Synchronous.  *out receives the plan. */
pst_status fft2d_plan(int nx, int ny, pst_kind kind, pst_prec prec, int batch,
                      void* hip_stream, pst_plan* out);

/* Bytes of device workspace the plan needs for every entry point below. */
pst_status pst_workspace_size(pst_plan plan, size_t* bytes);

/* Hand the plan caller-owned device memory of at least
 * pst_workspace_size() bytes (256-byte aligned).  Without this call the
 * plan allocates its own workspace on first use. */
pst_status pst_set_workspace(pst_plan plan, void* dev_ptr, size_t bytes);

/* 2D transform of every field of the batch.
 * C2C: in, out are [batch][ny][nx] complex; in == out is allowed.
 * R2C: sign -1 takes real [batch][ny][nx] to complex [batch][ny][nx/2+1];
 *      sign +1 takes complex [batch][ny][nx/2+1] (Hermitian half spectrum)
 *      to real [batch][ny][nx]; in must differ from out.
 * sign -1: forward, unnormalised; sign +1: inverse, scaled by 1/(nx*ny). */
pst_status fft2d_exec(pst_plan plan, const void* in, void* out, int sign);

/* Release the plan and everything it owns.  Synchronises its stream. */
pst_status fft2d_destroy(pst_plan plan);

/* --------------------------------------------------------------- solvers -- */

/* NLS, split-step Fourier (Section "A Numerical Method for the Nonlinear
 * Schrodinger Equation"): nsteps Strang steps L(dt/2) N(dt) L(dt/2) with
 * L the exact linear flow exp(-i |k|^2 t) in Fourier space and N the exact
 * nonlinear flow psi -> exp(-i g |psi|^2 dt) psi.  Adjacent half steps are
 * merged inside one call.  psi: C2C plan field, physical values in and out,
 * updated in place.  Needs a C2C plan. */
pst_status nls_step(pst_plan plan, void* psi, const pst_nls_params* p, int nsteps);

/* Sine-Gordon start-up: from u0 = u(0) and v0 = u_t(0) (real fields), write
 * u_prev = u^0 and u_curr = u^1, where u^1 solves the three-level scheme at
 * n = 0 with u^{-1} = u^1 - 2 dt v0 substituted.  Needs an R2C plan. */
pst_status sg_start(pst_plan plan, const void* u0, const void* v0, void* u_prev,
                    void* u_curr, const pst_sg_params* p);

/* Sine-Gordon (eq. sgmethodunformatted, Laplacian sign as in eq. sg):
 * advances the pair (u_prev, u_curr) = (u^{n-1}, u^n) by nsteps of
 *   (u^{n+1} - 2u^n + u^{n-1})/dt^2 - Delta (u^{n+1} + 2u^n + u^{n-1})/4
 *       = -sin u^n,
 * leaving (u^{n+nsteps-1}, u^{n+nsteps}) in (u_prev, u_curr).  Real fields,
 * R2C plan. */
pst_status sg_step(pst_plan plan, void* u_prev, void* u_curr, const pst_sg_params* p,
                   int nsteps);

/* sg_step for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * the same steps and results as sg_step, with the work arrays in a fixed
 * 64 MiB device array of the library (one per GPU, held until the process
 * ends) instead of the plan's workspace; calls no allocating routine.  The
 * plan's device must be current.  Its three half spectra need
 * 3 * batch * ny * (nx/2+1) complex values of the plan's precision (each
 * array rounded up to 256 bytes): up to 2048 x 2048 FP32 or 1024 x 1024
 * FP64 per field; PST_ERR_INVALID beyond 64 MiB.  Every call on one GPU
 * shares that array: calls that overlap on a GPU (other streams, other
 * threads) race; calls ordered on one stream do not.  Per-pass profiling
 * events are not recorded. */
pst_status sg_step_noalloc(pst_plan plan, void* u_prev, void* u_curr, const pst_sg_params* p,
                           int nsteps);

/* Navier-Stokes (Section "A Numerical Method for the 2D Navier-Stokes
 * Equation"): nsteps Crank-Nicolson steps, the Jacobian
 * J = psi_y omega_x - psi_x omega_y averaged between levels n and n+1 and
 * the n+1 level found by fixed-point iteration from omega^n.  The Jacobian's
 * spectrum is truncated to |m_x|, |m_y| <= floor((n-1)/3) (2/3 rule).
 * omega: real vorticity, updated in place; R2C plan.  If dev_iters is not
 * NULL it is a device int array of nsteps*batch entries receiving the
 * iterations taken by each step of each field.  A step that reaches
 * max_iter latches PST_ERR_NOT_CONVERGED (see pst_sync_status) and keeps
 * the last iterate. */
pst_status ns_step(pst_plan plan, void* omega, const pst_ns_params* p, int nsteps,
                   int* dev_iters);

/* Conserved quantities in double precision (FP64 accumulation on the
 * device, fixed summation order).  Synchronises the plan's stream and writes
 * 4 doubles per batch field to host array out[batch*4]:
 *   PST_NLS (eq. nlsmassenergy with coefficient g), f0 = psi, params =
 *     pst_nls_params: {mass, energy, kinetic, potential} with
 *     mass = integral |psi|^2, energy = integral |grad psi|^2/2 + g|psi|^4/4;
 *   PST_SG, f0 = u^n, f1 = u^{n+1}, params = pst_sg_params: staggered
 *     Hamiltonian H^{n+1/2} = integral (u_t^2 + |grad ubar|^2)/2 +
 *     ((1 - cos u^{n+1}) + (1 - cos u^n))/2 with u_t = (u^{n+1}-u^n)/dt and
 *     ubar = (u^{n+1}+u^n)/2:  {H, kinetic, gradient, potential};
 *   PST_NS, f0 = omega, params = pst_ns_params: {energy, enstrophy, 0, 0}
 *     with energy = integral |u|^2/2 and enstrophy = integral omega^2/2.
 * Integrals are dx*dy*sum; gradient terms use Parseval.  A non-finite
 * result returns PST_ERR_NONFINITE (the values are still written). */
pst_status conserved_quantities(pst_plan plan, pst_eq eq, const void* f0, const void* f1,
                                const void* params, double* out);

/* Device status latched since the last call (PST_OK,
 * PST_ERR_NOT_CONVERGED or PST_ERR_NONFINITE); clears it.  Synchronises. */
pst_status pst_sync_status(pst_plan plan, pst_status* device_status);

/* -------------------------------------------------------------- batching -- */

/* One simulation advanced by solve_batch.  f0/f1 are the caller's device
 * fields (256-byte aligned): NLS psi (f1 unused); SG (u_prev, u_curr); NS
 * omega (f1 unused).  params points to the equation's parameter struct.
 * dev_status, if not NULL, is a device int receiving this request's status
 * when the call's work completes: PST_ERR_NONFINITE if the field holds a
 * non-finite value at the end of a chunk of steps (or, for NS, a fixed-point
 * residual is not finite), else PST_ERR_NOT_CONVERGED if an NS step reached
 * max_iter, else PST_OK.  A failure already held in *dev_status (left by an
 * earlier call) is kept unless this call finds a worse one (NONFINITE
 * outranks NOT_CONVERGED); any other value is overwritten.  Zero it before
 * a simulation's first call. */
typedef struct {
  pst_eq eq;
  int nx, ny;
  pst_prec prec;
  int nsteps;
  const void* params;
  void* f0;
  void* f1;
  int* dev_status;
} pst_request;

/* Advance n independent simulations, each by its own nsteps, on
 * hip_stream (not a batched form of anything in the paper, whose programs
 * run one simulation each).  Requests are grouped by (equation, nx, ny,
 * precision, parameters); every group advances in one launch per pass
 * regardless of how many simulations it holds.  A request's result does not
 * depend on which other requests share the call, and one request's failure
 * (non-finite field, non-convergence) does not alter another's result.
 * Asynchronous on hip_stream, except that adaptive Navier-Stokes requests
 * (fixed_iters = 0) make the host wait once per step for the convergence
 * flags.  The library keeps one internal plan (tables and workspace) per
 * size class in use; see pst_batch_cache_bytes.  Errors in a request's
 * fields or parameters return PST_ERR_INVALID before anything is launched. */
pst_status solve_batch(const pst_request* reqs, int n, void* hip_stream);

/* Device bytes held by solve_batch's cached internal plans (workspace,
 * tables, status words), for callers that budget device memory. */
pst_status pst_batch_cache_bytes(size_t* bytes);

/* Release every cached internal plan of solve_batch (waits for their
 * streams); the next call recreates what it needs. */
pst_status pst_batch_cache_release(void);

/* ------------------------------------------------------------- utilities -- */

/* Message of the last error returned on the calling thread ("" if none). */
const char* pst_last_error(void);

/* Library version string. */
const char* pst_version(void);

/* Tile variants (not in the paper, which observed that launch parameters
 * chosen by the compiler ran 2x slower and that autotuning would help).
 *
 * Column passes (lines along y) run W adjacent columns per block.  Variant
 * 0, the default, exists for every length n: the widest W that fits 1024
 * threads and 150 KB of LDS, 16 values of a line per thread, complex values
 * exchanged through LDS between stages, radix 16.  For two-line passes
 * (sine-Gordon, Navier-Stokes, real transforms) and for single-field passes
 * shorter than 4096, variant 1 is half of variant 0's W; two-line passes of
 * lines of 512 and more add 2 and 3, a quarter and an eighth of it (those
 * that are at least 1).  Single-field
 * column passes (NLS steps and C2C transforms) of lines of 4096 and more add,
 * in FP32:
 *   1: the same W, 32 values per thread, real and imaginary parts exchanged
 *      one after the other ("split": half the threads and half the LDS);
 *   2: the same W, 16 values per thread, split, registers capped so that two
 *      1024-thread blocks fit a CU;
 *   3: twice the W, 32 values per thread, split;
 *   4: the same W, 16 values per thread, split, no register cap;
 * and in FP64:
 *   1: half of variant 0's W;
 *   2: variant 0's W, 32 values per thread, split;
 *   3: variant 0's W, 16 values per thread, split;
 *   4: twice variant 0's W, 16 values per thread, split (full 128-byte row
 *      segments);
 *   5: variant 0's W, radix 8 with 8 values per thread, split.
 * pst_column_variant_info reports (columns per block, values per thread,
 * split 0/1, radix) of variant for length n; single_field != 0 asks about
 * the single-field passes.  PST_ERR_INVALID if n is not a supported length
 * or the variant does not exist. */
pst_status pst_column_variant_info(pst_prec prec, int n, int variant, int single_field, int* columns,
                                   int* values_per_thread, int* split, int* radix);

/* Row variants of the NLS in-place row pass (the pass of every step; the
 * entry and exit passes keep the default).  Lines of 4096 and more run one
 * line per block: 0, 16 values per thread with the complex exchange (32
 * values, split, at 8192); 1, 16 values, split; 2, radix 8 with 8 values per
 * thread, split; 3, radix 8, complex exchange.  Shorter lines run row pairs,
 * P per block: 0, the default P (256 threads); then P/2 (where P >= 2) and
 * 2P (where it fits 1024 threads and 150 KB of LDS), numbered in that
 * order.  pst_row_variant_info
 * reports (row pairs per block, 0 for one line per block; values per thread;
 * split; radix).  Variants with the same radix and values per thread give
 * bit-identical results; the others differ by rounding. */
pst_status pst_row_variant_info(pst_prec prec, int n, int variant, int* pairs_per_block,
                                int* values_per_thread, int* split, int* radix);

/* Autotuning: times, on workspace data, the in-place row pass in each row
 * variant (NLS) and then the column pass of equation eq in each column
 * variant (for NLS one row pass in the chosen row variant and one column
 * pass per timed launch), each as the best of three windows of about 1 ms
 * of launches; keeps the fastest in the plan and remembers them for
 * later plans of the same (eq, precision, nx, ny) in this process, so that
 * every plan of that class runs the same variants.  Synchronises.  *chosen
 * (may be NULL) receives the column variant. */
pst_status pst_autotune(pst_plan plan, pst_eq eq, int* chosen);

/* Column variant used by this plan's column passes of length ny (0 by
 * default).  PST_ERR_INVALID if the variant does not exist for ny and the
 * plan's kind (C2C plans: single-field variants; R2C plans: two-line). */
pst_status pst_set_column_variant(pst_plan plan, int variant);

/* Row variant of this plan's NLS in-place row pass (0 by default; R2C
 * plans have only variant 0).  PST_ERR_INVALID if it does not exist. */
pst_status pst_set_row_variant(pst_plan plan, int variant);

/* The plan's current (row, column) variants. */
pst_status pst_get_variants(pst_plan plan, int* row_variant, int* column_variant);

/* Per-pass timing.  While enabled, every pass kernel that plan launches is
 * bracketed by a pair of HIP events recorded on the plan's stream.
 * pst_profile_read synchronises the stream and returns, for pass id
 * (PST_PASS_*), the summed duration in milliseconds and the number of
 * launches recorded since the last read or enable, then forgets them. */
typedef enum {
  PST_PASS_NLS_ROW = 0, PST_PASS_NLS_COL = 1, PST_PASS_SG_ROW = 2, PST_PASS_SG_COL = 3,
  PST_PASS_NS_ROW = 4, PST_PASS_NS_COL = 5, PST_PASS_COUNT = 6
} pst_pass;
pst_status pst_profile_enable(pst_plan plan, int enable);
pst_status pst_profile_read(pst_plan plan, int pass, double* total_ms, int* count);

#ifdef __cplusplus
}
#endif

#endif /* PST_H_ */
