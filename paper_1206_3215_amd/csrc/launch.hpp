// Host-side launchers of the pst kernels, called by the runtime (runtime.cpp).
// Each returns the HIP error of the launch; geometry and pointers are
// validated by the caller.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace pst {

enum Prec { P32 = 0, P64 = 1 };

// Status bits latched by kernels into a plan's device status word.
enum : int { ST_NONFINITE = 1, ST_NOT_CONVERGED = 2 };

// Column-pass tile: W adjacent columns per block, bounded by the block size
// and by the LDS footprint.
int col_tile_max(Prec p, int n);

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
// c2r: half spectra -> real rows, times scale.  Rows are processed in
// pairs; nlines may be odd.
hipError_t fft_row_r2c(Prec p, int n, int nlines, const void* in, void* out, const void* tw,
                       hipStream_t s);
hipError_t fft_row_c2r(Prec p, int n, int nlines, const void* in, void* out, double scale,
                       const void* tw, hipStream_t s);

// ----------------------------------------------------------------- NLS ---
// mode 0: H = nx * FFT_x(psi); 1: H <- FFT_x(e^{-i c |iFFT_x H|^2} iFFT_x H);
// 2: psi = iFFT_x(H) / nx.  phase_coef = g dt / nx^2, scale as stated.
hipError_t nls_row(Prec p, int nx, int nlines, void* psi, int mode, double phase_coef,
                   double scale, const void* tw, hipStream_t s);
// Column: FFT_y, multiply by ex[mx]*ey[my], iFFT_y (in place).
hipError_t nls_col(Prec p, int ny, int nx, int nfields, void* psi, const void* tw,
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

}  // namespace pst
