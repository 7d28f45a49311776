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

// UNI: all lines of a block lie in one field (always so when the field has
// at least LPB rows); the field is then reached through a buffer resource.
template <typename T, int N, int MODE, int VPT, bool SPLIT, bool UNI>
__global__ __launch_bounds__((RowGeom<T, N, VPT, SPLIT>::THREADS)) void k_nls_row(
    FieldRef psi, int nlines, int lny, T phase_coef, T scale, const cpx<T>* __restrict__ tw) {
  using G = RowGeom<T, N, VPT, SPLIT>;
  extern __shared__ char smem[];
  const int lid = threadIdx.x / G::TL, t = threadIdx.x % G::TL;
  const int line = blockIdx.x * G::LPB + lid;
  const bool valid = line < nlines;
  void* L = SPLIT ? (void*)(reinterpret_cast<T*>(smem) + lid * G::STRIDE)
                  : (void*)(reinterpret_cast<cpx<T>*>(smem) + lid * G::STRIDE);
  // lines past the end (a partial last block) recompute the last line and do not store
  const int lc = valid ? line : nlines - 1;
  const int ny = 1 << lny;
  cpx<T> v[G::R];
  auto body = [&]() {
    if constexpr (MODE == 0) {
      line_fft<N, false, 1, VPT, SPLIT>(v, L, t, tw);
#pragma unroll
      for (int s = 0; s < G::R; ++s) v[s] = v[s] * scale;
    } else if constexpr (MODE == 1) {
      line_fft<N, true, 1, VPT, SPLIT>(v, L, t, tw);
#pragma unroll
      for (int s = 0; s < G::R; ++s) v[s] = rotate_neg(v[s], phase_coef * norm2(v[s]));
      line_fft<N, false, 1, VPT, SPLIT>(v, L, t, tw);
    } else {
      line_fft<N, true, 1, VPT, SPLIT>(v, L, t, tw);
#pragma unroll
      for (int s = 0; s < G::R; ++s) v[s] = v[s] * scale;
    }
  };
  if constexpr (UNI) {
    const int f = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * G::LPB) >> lny);
    const FieldBuf fb(psi.at(f), (unsigned)((size_t)ny * N * sizeof(cpx<T>)));
    const unsigned o0 = (unsigned)((lc & (ny - 1)) * N + t) * (unsigned)sizeof(cpx<T>);
    constexpr unsigned ds = G::TL * sizeof(cpx<T>);
#pragma unroll
    for (int s = 0; s < G::R; ++s) v[s] = fb.template ldc<T>(o0, s * ds);
    body();
    if (valid) {
#pragma unroll
      for (int s = 0; s < G::R; ++s) fb.st(o0, s * ds, v[s]);
    }
  } else {
    gptr<cpx<T>> g = field<cpx<T>>(psi, lc >> lny) + (size_t)(lc & (ny - 1)) * N;
#pragma unroll
    for (int s = 0; s < G::R; ++s) v[s] = gload(g + (t + s * G::TL));
    body();
    if (valid) {
#pragma unroll
      for (int s = 0; s < G::R; ++s) gstore(g + (t + s * G::TL), v[s]);
    }
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

// Row configuration: 32 values per thread with the split exchange for FP32
// lines of 8192 (256 threads and 35 KB of LDS per line, so several lines
// share a CU); 16 values per thread and the complex exchange otherwise.
template <typename T, int N>
struct NlsRowCfg {
  static constexpr bool BIG = std::is_same<T, float>::value && N >= 8192;
  static constexpr int VPT = BIG ? 32 : line_radix(N);
  static constexpr bool SPLIT = BIG;
};

template <typename T, int N, int MODE, bool UNI>
static void launch_row(int nlines, int ny, FieldRef psi, double pc, double scale, const void* tw, hipStream_t s) {
  using C = NlsRowCfg<T, N>;
  using G = RowGeom<T, N, C::VPT, C::SPLIT>;
  auto* k = &k_nls_row<T, N, MODE, C::VPT, C::SPLIT, UNI>;
  allow_lds(k, G::LDS_BYTES);
  hipLaunchKernelGGL(k, dim3((nlines + G::LPB - 1) / G::LPB), dim3(G::THREADS), G::LDS_BYTES, s, psi, nlines,
                     ilog2c(ny), (T)pc, (T)scale, (const cpx<T>*)tw);
}

template <typename T>
static hipError_t row(int nx, int nlines, int ny, FieldRef psi, int mode, double pc, double scale,
                      const void* tw, hipStream_t s) {
  bool ok = dispatch_n(nx, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    using C = NlsRowCfg<T, N>;
    constexpr int LPB = RowGeom<T, N, C::VPT, C::SPLIT>::LPB;
    const bool uni = LPB == 1 || ny >= LPB;
    auto go = [&](auto m) {
      constexpr int MODE = decltype(m)::value;
      if (uni) launch_row<T, N, MODE, true>(nlines, ny, psi, pc, scale, tw, s);
      else launch_row<T, N, MODE, false>(nlines, ny, psi, pc, scale, tw, s);
    };
    if (mode == 0) go(IntC<0>{});
    else if (mode == 1) go(IntC<1>{});
    else go(IntC<2>{});
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
