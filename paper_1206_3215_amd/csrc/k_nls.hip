// NLS split-step passes (Section "A Numerical Method for the Nonlinear
// Schrodinger Equation").
//
// Between passes the field is held as H = FFT_x(psi): transformed along x
// only.  Because the 2D transform factorises, one time step is two sweeps:
//   row pass:    psi = iFFT_x(H);  psi *= exp(-i g |psi|^2 dt);  H = FFT_x(psi)
//   column pass: psi_hat = FFT_y(H); psi_hat *= E_x[mx] E_y[my]; H = iFFT_y(psi_hat)
// with E = exp(-i k^2 tau) separable in x and y.  Adjacent linear half steps
// of consecutive Strang steps merge into one full step, so a call of n steps
// is: entry row (FFT_x only), column (half), n-1 x [row, column (full)],
// row, column (half), exit row (iFFT_x only).  The unnormalised transforms'
// factors go into the phase coefficient and one scaling in the column pass.
// The propagator tables hold E - 1 = (cos - 1, -sin): multiplying as
// v + v (E - 1) keeps |E| = 1 to within rounding of the small correction;
// rounded (cos, -sin) pairs carry a bias of |E| near 1 for the energetic
// low modes that would drain or feed the mass at every step.
#include "kernels.hpp"
#include "launch.hpp"

namespace pst {

template <typename T, int N, int MODE>
__global__ __launch_bounds__((RowGeom<T, N>::THREADS)) void k_nls_row(
    FieldRef psi, int nlines, int lny, T phase_coef, T scale, const cpx<T>* __restrict__ tw) {
  using G = RowGeom<T, N>;
  extern __shared__ char smem[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem);
  const int lid = threadIdx.x / G::TL, t = threadIdx.x % G::TL;
  const int line = blockIdx.x * G::LPB + lid;
  const bool valid = line < nlines;
  cpx<T>* L = lds + lid * lds_line_stride<T>(N);
  // lines past the end (a partial last block) recompute the last line and do not store
  const int lc = valid ? line : nlines - 1;
  gptr<cpx<T>> g = field<cpx<T>>(psi, lc >> lny) + (size_t)(lc & ((1 << lny) - 1)) * N;
  cpx<T> v[G::R];
#pragma unroll
  for (int s = 0; s < G::R; ++s) v[s] = gload(g + (t + s * G::TL));
  if constexpr (MODE == 0) {
    line_fft<N, false>(v, L, t, tw);
#pragma unroll
    for (int s = 0; s < G::R; ++s) v[s] = v[s] * scale;
  } else if constexpr (MODE == 1) {
    line_fft<N, true>(v, L, t, tw);
#pragma unroll
    for (int s = 0; s < G::R; ++s) v[s] = rotate_neg(v[s], phase_coef * norm2(v[s]));
    line_fft<N, false>(v, L, t, tw);
  } else {
    line_fft<N, true>(v, L, t, tw);
#pragma unroll
    for (int s = 0; s < G::R; ++s) v[s] = v[s] * scale;
  }
  if (valid) {
#pragma unroll
    for (int s = 0; s < G::R; ++s) gstore(g + (t + s * G::TL), v[s]);
  }
}

template <typename T, int N, int WT, int VPT, bool SPLIT, int WPE>
__global__ __launch_bounds__((WT * (N / VPT))) __attribute__((amdgpu_waves_per_eu(WPE))) void k_nls_col(
    FieldRef psi, int nx, int tiles_per_field, const cpx<T>* __restrict__ tw, const cpx<T>* __restrict__ ex,
    const cpx<T>* __restrict__ ey, T scale) {
  using G = ColGeom<T, N, WT, VPT, SPLIT>;
  extern __shared__ char smem[];
  const int c = threadIdx.x % WT, t = threadIdx.x / WT;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int fld = tile / tiles_per_field;
  const int col = (tile % tiles_per_field) * WT + c;
  const bool valid = col < nx;
  const int cc = valid ? col : nx - 1;  // columns past the end recompute the last one, unstored
  const FieldBuf fb(psi.at(fld), (unsigned)((size_t)N * nx * sizeof(cpx<T>)));
  const unsigned o0 = (unsigned)(cc + t * nx) * (unsigned)sizeof(cpx<T>);
  const unsigned ds = (unsigned)(G::TL * nx) * (unsigned)sizeof(cpx<T>);  // row step of value s
  void* L = SPLIT ? (void*)(reinterpret_cast<T*>(smem) + c) : (void*)(reinterpret_cast<cpx<T>*>(smem) + c);
  cpx<T> v[G::R];
#pragma unroll
  for (int s = 0; s < G::R; ++s) v[s] = fb.template ldc<T>(o0, s * ds);
  line_fft<N, false, WT, VPT, SPLIT>(v, L, t, tw);
  // the propagator loads are issued after the forward transform: hoisted
  // above it they would hold registers through the whole transform
  asm volatile("" ::: "memory");
  const cpx<T> exm = ex[cc];
#pragma unroll
  for (int s = 0; s < G::R; ++s) {
    const cpx<T> w = v[s] * scale;
    const cpx<T> wx = w + cmul(w, exm);
    v[s] = wx + cmul(wx, ey[t + s * G::TL]);
  }
  line_fft<N, true, WT, VPT, SPLIT>(v, L, t, tw);
  if (valid) {
#pragma unroll
    for (int s = 0; s < G::R; ++s) fb.st(o0, s * ds, v[s]);
  }
}

template <typename T>
static hipError_t row(int nx, int nlines, int ny, FieldRef psi, int mode, double pc, double scale,
                      const void* tw, hipStream_t s) {
  bool ok = dispatch_n(nx, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    using G = RowGeom<T, N>;
    const int grid = (nlines + G::LPB - 1) / G::LPB;
    if (mode == 0) {
      allow_lds((k_nls_row<T, N, 0>), G::LDS_BYTES);
      hipLaunchKernelGGL((k_nls_row<T, N, 0>), dim3(grid), dim3(G::THREADS), G::LDS_BYTES, s,
                         psi, nlines, ilog2c(ny), (T)pc, (T)scale, (const cpx<T>*)tw);
    } else if (mode == 1) {
      allow_lds((k_nls_row<T, N, 1>), G::LDS_BYTES);
      hipLaunchKernelGGL((k_nls_row<T, N, 1>), dim3(grid), dim3(G::THREADS), G::LDS_BYTES, s,
                         psi, nlines, ilog2c(ny), (T)pc, (T)scale, (const cpx<T>*)tw);
    } else {
      allow_lds((k_nls_row<T, N, 2>), G::LDS_BYTES);
      hipLaunchKernelGGL((k_nls_row<T, N, 2>), dim3(grid), dim3(G::THREADS), G::LDS_BYTES, s,
                         psi, nlines, ilog2c(ny), (T)pc, (T)scale, (const cpx<T>*)tw);
    }
  });
  return ok ? hipGetLastError() : hipErrorInvalidValue;
}

hipError_t nls_row(Prec p, int nx, int nlines, int ny, FieldRef psi, int mode, double phase_coef, double scale,
                   const void* tw, hipStream_t s) {
  return p == P32 ? row<float>(nx, nlines, ny, psi, mode, phase_coef, scale, tw, s)
                  : row<double>(nx, nlines, ny, psi, mode, phase_coef, scale, tw, s);
}

template <typename T>
static hipError_t col(int ny, int nx, int nfields, FieldRef psi, const void* tw, const void* ex,
                      const void* ey, int W, hipStream_t s) {
  bool ok = false;
  dispatch_n(ny, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    ok = dispatch_col1<T, N>(W, [&](auto cfg) {
      using C = decltype(cfg);
      using G = ColGeom<T, N, C::w, C::vpt, C::split>;
      const int tiles = (nx + C::w - 1) / C::w;
      auto* k = &k_nls_col<T, N, C::w, C::vpt, C::split, C::wpe>;
      allow_lds(k, G::LDS_BYTES);
      hipLaunchKernelGGL(k, dim3(tiles * nfields), dim3(G::THREADS), G::LDS_BYTES, s, psi, nx, tiles,
                         (const cpx<T>*)tw, (const cpx<T>*)ex, (const cpx<T>*)ey, (T)(1.0 / ((double)nx * N)));
    });
  });
  return ok ? hipGetLastError() : hipErrorInvalidValue;
}

hipError_t nls_col(Prec p, int ny, int nx, int nfields, FieldRef psi, const void* tw, const void* ex,
                   const void* ey, int W, hipStream_t s) {
  return p == P32 ? col<float>(ny, nx, nfields, psi, tw, ex, ey, W, s)
                  : col<double>(ny, nx, nfields, psi, tw, ex, ey, W, s);
}

}  // namespace pst
