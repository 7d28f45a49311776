// Host-side launchers of the pst kernels, called by the runtime (runtime.cpp).
// Each returns the HIP error of the launch; geometry and pointers are
// validated by the caller.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace pst {

enum Prec { P32 = 0, P64 = 1 };

// Addressing of caller fields: field f starts at table[f] when a device
// pointer table is given, else at base + f * stride bytes.  Used for every
// field the solver entry points take from the caller, so that a launch can
// advance simulations whose fields are not contiguous (batched requests).
struct FieldRef {
  char* base = nullptr;
  long long stride = 0;
  void* const* table = nullptr;
  __host__ __device__ char* at(int f) const { return table ? (char*)table[f] : base + f * stride; }
};
inline FieldRef contiguous(const void* p, size_t field_bytes) {
  FieldRef r;
  r.base = (char*)p;
  r.stride = (long long)field_bytes;
  return r;
}

// Status bits latched by kernels into a plan's device status word.
enum : int { ST_NONFINITE = 1, ST_NOT_CONVERGED = 2 };

// Where a kernel latches a status bit: the plan-wide word and, for batched
// requests, a per-field word reached through a device pointer table (either
// may be NULL; so may a table entry).
struct StatusRef {
  int* plan = nullptr;
  int* const* field = nullptr;
};

// Column tile variant `var` for lines of length n: columns per block,
// values per thread, split exchange, radix.  single: a single-field pass
// (NLS, C2C); two-line passes have no split or radix variants.  False if
// not compiled.
bool col_variant_info(Prec p, int n, int var, bool single, int* w, int* vpt, int* split, int* radix);
// Row variant `var` of the NLS in-place row pass for lines of length n: row
// pairs per block (0: one line per block), values per thread, split
// exchange, radix.  False if not compiled.
bool nls_row_variant_info(Prec p, int n, int var, int* pairs, int* vpt, int* split, int* radix);

// ------------------------------------------------------- mixed radix ---
// Stage list of the line FFT of a length n = 2^a 3^b 5^c that is not a
// power of two (k_mixed.hip): radix r[s] of stage s, the product ns[s] of
// the earlier radices, and the offset toff[s] of its (r-1) ns entries in the
// length's twiddle table (entry (q-1) ns + k = exp(-2 pi i q k / (ns r))).
struct MixedLine {
  int n = 0, nst = 0;
  int r[14] = {}, ns[14] = {}, toff[14] = {};
};
// Whether a mixed-radix line of length n fits the passes' LDS (two buffers
// of n complex values: FP32 up to 9600, FP64 up to 4800).
bool mixed_supported(Prec p, int n);
// C2C rows (nlines contiguous lines) and columns ([field][n][ld], first
// ncols columns), times scale; in may equal out.
hipError_t mixed_row_c2c(Prec p, const MixedLine& ml, int nlines, const void* in, void* out, bool inv,
                         double scale, const void* tw, hipStream_t s);
hipError_t mixed_col_c2c(Prec p, const MixedLine& ml, int ncols, int ld, int nfields, const void* src, void* dst,
                         bool inv, double scale, const void* tw, hipStream_t s);
// Real rows of length n: forward to the n/2+1 half spectrum, inverse from it
// (times scale).
hipError_t mixed_row_r2c(Prec p, const MixedLine& ml, int nlines, const void* in, void* out, const void* tw,
                         hipStream_t s);
hipError_t mixed_row_c2r(Prec p, const MixedLine& ml, int nlines, const void* in, void* out, double scale,
                         const void* tw, hipStream_t s);
// NLS passes with nls_row / nls_col semantics on plain rows (no pair
// layout); fields of ny rows of ml.n (row pass) or nx (column pass).
hipError_t mixed_nls_row(Prec p, const MixedLine& ml, int nlines, int ny, FieldRef psi, int mode,
                         double phase_coef, double scale, const void* tw, hipStream_t s, StatusRef st);
hipError_t mixed_nls_col(Prec p, const MixedLine& ml, int nx, int nfields, FieldRef psi, const void* tw,
                         const void* ex, const void* ey, hipStream_t s);
// NLS diagnostics partials in nls_cq_row / nls_cq_col layout (spec: FFT_x
// then FFT_y of psi in place), for nls_cq_finish.
hipError_t mixed_nls_cq(Prec p, const MixedLine& mlx, const MixedLine& mly, int nfields, const void* psi,
                        void* spec, double* row_part, double* col_part, const void* twx, const void* twy,
                        double kx0, double ky0, hipStream_t s);

// ----------------------------------------------------------------- FFT ---
// Row pass over nlines contiguous complex lines of length n: out = FFT(in)
// (inverse if inv), times scale.  in may equal out.
hipError_t fft_row_c2c(Prec p, int n, int nlines, const void* in, void* out, bool inv,
                       double scale, const void* tw, hipStream_t s);
// Column pass: nfields fields of ny rows, each row ld complex elements of
// which the first ncols are transformed (columns of length ny), times
// scale; src may equal dst.
hipError_t fft_col_c2c(Prec p, int ny, int ncols, int ld, int nfields, const void* src, void* dst,
                       bool inv, double scale, const void* tw, int W, hipStream_t s);

// Real rows.  r2c: nlines real rows of length n -> half spectra (n/2+1).
// c2r: half spectra -> real rows, times scale (rows of a field f with
// skip[f] != 0 are not stored; skip may be NULL).  Rows are processed in
// pairs; nlines may be odd.
// The real side is a FieldRef of fields with ny rows (ny a power of two).
hipError_t fft_row_r2c(Prec p, int n, int nlines, int ny, FieldRef in, void* out, const void* tw,
                       hipStream_t s);
hipError_t fft_row_c2r(Prec p, int n, int nlines, int ny, const void* in, FieldRef out, double scale,
                       const void* tw, hipStream_t s, const int* skip = nullptr);

// ----------------------------------------------------------------- NLS ---
// mode 0: H = nx * FFT_x(psi); 1: H <- FFT_x(e^{-i c |iFFT_x H|^2} iFFT_x H);
// 2: psi = iFFT_x(H) / nx.  phase_coef = g dt / nx^2, scale as stated.
// Mode 2 latches ST_NONFINITE into st for a field whose result holds a
// non-finite value.  var selects the row variant of mode 1.
hipError_t nls_row(Prec p, int nx, int nlines, int ny, FieldRef psi, int mode, double phase_coef,
                   double scale, const void* tw, hipStream_t s, StatusRef st = StatusRef(), int var = 0);
// Column: FFT_y, multiply by (1 + ex[mx]) (1 + ey[my]) / (nx ny), iFFT_y (in place).
hipError_t nls_col(Prec p, int ny, int nx, int nfields, FieldRef psi, const void* tw,
                   const void* ex, const void* ey, int W, hipStream_t s);

// ------------------------------------------------------- reductions ---
// NLS diagnostics.  Row: spec = FFT_x(psi), line sums of |psi|^2, |psi|^4
// into part[line*2 + {0,1}].  Column: FFT_y of spec (in place) and line sums
// of |k|^2 |psi_hat|^2 into part[col] (col = field*nx + mx).
hipError_t nls_cq_row(Prec p, int nx, int nlines, const void* psi, void* spec,
                      double* part, const void* tw, hipStream_t s);
hipError_t nls_cq_col(Prec p, int ny, int nx, int nfields, void* spec, double* part,
                      const void* tw, double kx0, double ky0, int W, hipStream_t s);
// Combine line partials (fixed order) into out[f*4 + 0..3] for each field f
// and latch PST_ERR_NONFINITE into *status if a result is not finite.
hipError_t nls_cq_finish(int nfields, int ny, int nx, const double* row_part,
                         const double* col_part, double dxdy, double kin_coef, double g,
                         double* out, int* status, hipStream_t s);

// ------------------------------------------------------------------ SG ---
// Row pass over row pairs (increment form, see k_sg.hip):
//   mode 0 (entry): U, S = 2 R2C_x(u_old), 2 R2C_x(sin u_old); if d_out is
//                   not NULL, d_out = u_old - d_old.
//   mode 1 (step):  d_out = d_old + C2R_x(W); u_out = u_old + d_out; U, S.
//   mode 2 (final): d = alpha d_old + C2R_x(W); u_out = u_old + d;
//                   prev_out = u_old; ST_NONFINITE latched into st for a
//                   field whose u_out holds a non-finite value.
// Each element is read before it is written, so outputs may alias inputs.
hipError_t sg_row(Prec p, int mode, int nx, int nlines, int ny, const void* W, FieldRef u_old, FieldRef d_old,
                  double alpha, FieldRef u_out, FieldRef d_out, FieldRef prev_out, void* U, void* S,
                  const void* tw, hipStream_t s, StatusRef st = StatusRef());
// Column pass: W = iFFT_y(c1m FFT_y(U) - c2 FFT_y(S)) with a = |k|^2 dt2q,
// c1m = -2 cnum a/(1+a) sc, c2 = c2num/(1+a) sc.
hipError_t sg_col(Prec p, int ny, int nx, int nfields, const void* U, const void* S, void* W, const void* tw,
                  double kx0, double ky0, double dt2q, double cnum, double c2num, double sc, int Wt,
                  hipStream_t s);
// Hamiltonian H^{n+1/2}(f0 = u^n, f1 = u^{n+1}).
hipError_t sg_h_row(Prec p, int nx, int nlines, const void* f0, const void* f1, void* UB, double* part,
                    double inv_dt, const void* tw, hipStream_t s);
hipError_t sg_h_col(Prec p, int ny, int nx, int nfields, void* UB, double* part, const void* tw, double kx0,
                    double ky0, int Wt, hipStream_t s);
hipError_t sg_h_finish(int nfields, int npairs, int ncols, const double* row_part, const double* col_part,
                       double dxdy, double grad_coef, double* out, int* status, hipStream_t s);

// ------------------------------------------------------------------ NS ---
struct NsPtrs {
  const void* NH;  // Jacobian hybrid (times 2), or omega's x-transform at entry
  void* WN;        // w^n spectrum
  void* Q;         // -2h w^n - dt/2 N(w^n)
  void* DK;        // increment d^k = w^k - w^n
  void* D;         // 4 derivative hybrids, dstride complex apart
  size_t dstride;
  void* OUT;       // exit: iFFT_y(w^n + d) hybrid
  double* part;    // 2 doubles per column: residual, |w|^2
};
struct NsScalars {
  double kx0, ky0, hnu, qdt, nscale, dscale;
  int nx, kx_cut, ky_cut;
};
// Row pass: Jacobian of the derivative hybrids -> NH.  Blocks whose fields
// are all done (done != NULL) return at once.
hipError_t ns_row(Prec p, int nx, int nlines, int ny, const void* D, size_t dstride, void* NH, const int* done,
                  const void* tw, hipStream_t s);
// Column pass, mode 0 entry / 1 first iteration / 2 later iteration / 3 exit.
// Fields whose gate word is nonzero (gate may be NULL) are skipped.
hipError_t ns_col(Prec p, int mode, int ny, int nfields, const NsPtrs& P, const NsScalars& S, const int* gate,
                  const void* tw, int Wt, hipStream_t s);
// Iterations queued ahead of the host (see k_ns_finish): per-field park
// flags, the step each parked field stopped in, the most iterations a
// converged step took, whether this is the step's last queued iteration,
// and the step's index in the chunk.  park == NULL: the host polls instead.
struct NsPark {
  int* park = nullptr;
  int* park_step = nullptr;
  int* maxit = nullptr;
  int last = 0, step = 0;
};
// Convergence bookkeeping per field (see k_ns_finish); fstat, if not NULL,
// holds a per-field pointer receiving that field's ST_ bits.
hipError_t ns_finish(int nfields, int ncols, const double* part, double vol, double tol, double fp_floor,
                     int max_iter, int fixed, int first, int* done, int* iters, int* iters_out, double* resid,
                     int* status, int* const* fstat, const NsPark& pk, hipStream_t s);
// p[0..n) = v (a kernel, so that it may sit in a captured graph).
hipError_t fill_int(int* p, int n, int v, hipStream_t s);
// Diagnostics from omega's x-transform XH: energy and enstrophy.
hipError_t ns_cq_col(Prec p, int ny, int nx, int nfields, const void* XH, double* part, double kx0, double ky0,
                     const void* tw, int Wt, hipStream_t s);
hipError_t ns_cq_finish(int nfields, int ncols, const double* part, double en_coef, double zz_coef, double* out,
                        int* status, hipStream_t s);

}  // namespace pst
