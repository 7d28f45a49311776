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
// H is stored with the rows of each pair (2p, 2p+1) interleaved element by
// element: H(y, x) sits at (y - y%2) nx + 2x + y%2.  A row pass block owns
// whole pairs (the first pass reads psi's plain rows, the last writes them
// back), and a column pass block of W columns then reads and writes
// 2W-element (64-byte for W = 4, FP32) segments instead of W-element ones.
// The propagator tables hold E - 1 = (cos - 1, -sin): multiplying as
// v + v (E - 1) keeps |E| = 1 to within rounding of the small correction;
// rounded (cos, -sin) pairs carry a bias of |E| near 1 for the energetic
// low modes that would drain or feed the mass at every step.
#include "kernels.hpp"
#include "launch.hpp"

namespace pst {

// Row pass over row pairs: P pairs per block, the two rows of a pair on
// alternate lanes (l = lane & 1) and interleaved in LDS like a two-column
// tile.  MODE 0 reads plain rows of psi, MODE 2 writes them; everything else
// is in the pair-interleaved layout.  UNI: all pairs of a block lie in one
// field, reached through a buffer resource.
template <typename T, int N, int VPT, bool SPLIT, int P_ = 0>
struct PairGeom {
  static constexpr int R = VPT;
  static constexpr int TL = N / VPT;
  static constexpr int P = P_ > 0 ? P_ : TL >= 128 ? 1 : 128 / TL;
  static constexpr int THREADS = 2 * P * TL;
  static constexpr int LINE = lds_line_len(N);
  static constexpr size_t LDS_BYTES = (size_t)P * 2 * LINE * (SPLIT ? sizeof(T) : sizeof(cpx<T>));
};

template <typename T, int N, int MODE, int VPT, bool SPLIT, bool UNI, int P_>
__global__ __launch_bounds__((PairGeom<T, N, VPT, SPLIT, P_>::THREADS)) void k_nls_row(
    FieldRef psi, int npairs, int lny, T phase_coef, T scale, const cpx<T>* __restrict__ tw, StatusRef st) {
  using G = PairGeom<T, N, VPT, SPLIT, P_>;
  extern __shared__ char smem[];
  const int l = threadIdx.x & 1, q = threadIdx.x >> 1;
  const int t = q % G::TL, pl = q / G::TL;
  const int pair = blockIdx.x * G::P + pl;
  const bool valid = pair < npairs;
  // pairs past the end (a partial last block) recompute the last pair and do not store
  const int pc = valid ? pair : npairs - 1;
  const int ny = 1 << lny;
  const int r = (2 * pc) & (ny - 1);  // first row of the pair within its field
  const size_t slot0 = (size_t)pl * 2 * G::LINE + l;
  void* L = SPLIT ? (void*)(reinterpret_cast<T*>(smem) + slot0) : (void*)(reinterpret_cast<cpx<T>*>(smem) + slot0);
  cpx<T> v[G::R];
  auto body = [&]() {
    if constexpr (MODE == 0) {
      line_fft<N, false, 2, VPT, SPLIT>(v, L, t, tw);
#pragma unroll
      for (int s = 0; s < G::R; ++s) v[s] = v[s] * scale;
    } else if constexpr (MODE == 1) {
      line_fft<N, true, 2, VPT, SPLIT>(v, L, t, tw);
#pragma unroll
      for (int s = 0; s < G::R; ++s) v[s] = rotate_neg(v[s], phase_coef * norm2(v[s]));
      line_fft<N, false, 2, VPT, SPLIT>(v, L, t, tw);
    } else {
      line_fft<N, true, 2, VPT, SPLIT>(v, L, t, tw);
#pragma unroll
      for (int s = 0; s < G::R; ++s) v[s] = v[s] * scale;
    }
  };
  // element offsets of value s: plain row r + l, or the interleaved pair
  const unsigned plain0 = (unsigned)((r + l) * N + t), inter0 = (unsigned)(r * N + 2 * t + l);
  constexpr unsigned plain_ds = G::TL, inter_ds = 2 * G::TL;
  constexpr bool in_plain = MODE == 0, out_plain = MODE == 2;
  const unsigned i0 = in_plain ? plain0 : inter0, o0 = out_plain ? plain0 : inter0;
  const unsigned ids = in_plain ? plain_ds : inter_ds, ods = out_plain ? plain_ds : inter_ds;
  constexpr unsigned sz = sizeof(cpx<T>);
  // the exit pass reports a field holding a non-finite value
  auto check = [&](int f, bool uniform) {
    if constexpr (MODE == 2) {
      bool bad = false;
#pragma unroll
      for (int s = 0; s < G::R; ++s) bad = bad || !finite_c(v[s]);
      latch_nonfinite(bad && valid, st, f, uniform);
    }
  };
  if constexpr (UNI) {
    const int f = __builtin_amdgcn_readfirstlane((int)(2 * blockIdx.x * G::P) >> lny);
    const FieldBuf fb(psi.at(f), (unsigned)((size_t)ny * N * sz));
#pragma unroll
    for (int s = 0; s < G::R; ++s) v[s] = fb.template ldc<T>(i0 * sz, s * ids * sz);
    body();
    if (valid) {
#pragma unroll
      for (int s = 0; s < G::R; ++s) fb.st(o0 * sz, s * ods * sz, v[s]);
    }
    check(f, true);
  } else {
    const int f = (2 * pc) >> lny;
    gptr<cpx<T>> g = field<cpx<T>>(psi, f);
#pragma unroll
    for (int s = 0; s < G::R; ++s) v[s] = gload(g + (i0 + s * ids));
    body();
    if (valid) {
#pragma unroll
      for (int s = 0; s < G::R; ++s) gstore(g + (o0 + s * ods), v[s]);
    }
    // a wave spans 64/TL rows of whole pairs, all in one field when ny >= 64/TL
    check(f, ny * G::TL >= 64);
  }
}

template <typename T, int N, int WT, int VPT, bool SPLIT, int WPE, int R>
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
  // H(y, cc) of the pair-interleaved layout, y = t + s TL: for even TL the
  // pair parity of y is that of t (a uniform step per s), for TL = 1 (lines
  // of 16 or less) it is that of s
  constexpr bool EVEN = G::TL % 2 == 0;
  constexpr unsigned sz = sizeof(cpx<T>);
  const unsigned o0 = (unsigned)((t & ~1) * nx + 2 * cc + (t & 1)) * sz;
  const unsigned ds = (unsigned)(G::TL * nx) * sz;  // row step of value s
  // (per-lane, uniform) byte offsets of value s
  auto voff = [&](int s) { return EVEN ? o0 : (unsigned)((s & ~1) * nx + 2 * cc + (s & 1)) * sz; };
  auto soff = [&](int s) { return EVEN ? s * ds : 0u; };
  void* L = SPLIT ? (void*)(reinterpret_cast<T*>(smem) + c) : (void*)(reinterpret_cast<cpx<T>*>(smem) + c);
  cpx<T> v[G::R];
#pragma unroll
  for (int s = 0; s < G::R; ++s) v[s] = fb.template ldc<T>(voff(s), soff(s));
  line_fft<N, false, WT, VPT, SPLIT, R>(v, L, t, tw);
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
  line_fft<N, true, WT, VPT, SPLIT, R>(v, L, t, tw);
  if (valid) {
#pragma unroll
    for (int s = 0; s < G::R; ++s) fb.st(voff(s), soff(s), v[s]);
  }
}

// Long lines (N/VPT >= 256 threads), in-place pass (MODE 1): one line per
// block over the pair layout; line y reads every other element of its
// pair's span.  Blocks are
// mapped to lines so that each XCD takes a contiguous range of lines: the
// two lines of a pair run side by side on one XCD and share its L2.
template <typename T, int N, int MODE, int VPT, bool SPLIT, int R>
__global__ __launch_bounds__((N / VPT)) void k_nls_row1(FieldRef psi, int lny, T phase_coef, T scale,
                                                         const cpx<T>* __restrict__ tw) {
  constexpr int TL = N / VPT;
  extern __shared__ char smem[];
  const int t = threadIdx.x;
  const int line = xcd_tile(blockIdx.x, gridDim.x);
  const int ny = 1 << lny;
  const int y = line & (ny - 1), l = y & 1, r = y - l;
  void* L = smem;
  cpx<T> v[VPT];
  const unsigned plain0 = (unsigned)(y * N + t), inter0 = (unsigned)(r * N + 2 * t + l);
  constexpr bool in_plain = MODE == 0, out_plain = MODE == 2;
  const unsigned i0 = in_plain ? plain0 : inter0, o0 = out_plain ? plain0 : inter0;
  constexpr unsigned ids = in_plain ? TL : 2 * TL, ods = out_plain ? TL : 2 * TL;
  constexpr unsigned sz = sizeof(cpx<T>);
  const FieldBuf fb(psi.at(line >> lny), (unsigned)((size_t)ny * N * sz));
#pragma unroll
  for (int s = 0; s < VPT; ++s) v[s] = fb.template ldc<T>(i0 * sz, s * ids * sz);
  if constexpr (MODE == 0) {
    line_fft<N, false, 1, VPT, SPLIT, R>(v, L, t, tw);
#pragma unroll
    for (int s = 0; s < VPT; ++s) v[s] = v[s] * scale;
  } else if constexpr (MODE == 1) {
    line_fft<N, true, 1, VPT, SPLIT, R>(v, L, t, tw);
#pragma unroll
    for (int s = 0; s < VPT; ++s) v[s] = rotate_neg(v[s], phase_coef * norm2(v[s]));
    line_fft<N, false, 1, VPT, SPLIT, R>(v, L, t, tw);
  } else {
    line_fft<N, true, 1, VPT, SPLIT, R>(v, L, t, tw);
#pragma unroll
    for (int s = 0; s < VPT; ++s) v[s] = v[s] * scale;
  }
#pragma unroll
  for (int s = 0; s < VPT; ++s) fb.st(o0 * sz, s * ods * sz, v[s]);
}

// Row configuration: 32 values per thread with the split exchange for lines
// of 8192 (a pair then takes 512 threads and 70 KB (FP32) or 139 KB (FP64)
// of LDS); 16 values per thread and the complex exchange otherwise.
template <typename T, int N>
struct NlsRowCfg {
  static constexpr bool BIG = N >= 8192;
  static constexpr int VPT = BIG ? 32 : line_radix(N);
  static constexpr bool SPLIT = BIG;
};

template <typename T, int N, int MODE, bool UNI, int VPT, bool SPLIT, int P>
static void launch_row(int npairs, int ny, FieldRef psi, double pc, double scale, const void* tw, hipStream_t s,
                       StatusRef st) {
  using G = PairGeom<T, N, VPT, SPLIT, P>;
  auto* k = &k_nls_row<T, N, MODE, VPT, SPLIT, UNI, P>;
  allow_lds(k, G::LDS_BYTES);
  hipLaunchKernelGGL(k, dim3((npairs + G::P - 1) / G::P), dim3(G::THREADS), G::LDS_BYTES, s, psi, npairs,
                     ilog2c(ny), (T)pc, (T)scale, (const cpx<T>*)tw, st);
}

// Row pass of mode 0 (entry), 1 (the in-place step pass, in row variant
// var) or 2 (exit).  The entry and exit passes convert between layouts, so a
// pair's two rows must be owned by one block: they run the pair kernel in
// its default configuration (32 values per thread and the split exchange
// for lines of 8192).
template <typename T>
static hipError_t row(int nx, int nlines, int ny, FieldRef psi, int mode, double pc, double scale,
                      const void* tw, hipStream_t s, StatusRef st, int var) {
  if (ny % 2 != 0 || nlines % 2 != 0) return hipErrorInvalidValue;
  bool ok = false;
  dispatch_n(nx, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    using C = NlsRowCfg<T, N>;
    auto pairs = [&](auto m, auto cfg) {
      constexpr int MODE = decltype(m)::value;
      using RC = decltype(cfg);
      constexpr int P = PairGeom<T, N, RC::vpt, RC::split, RC::pairs>::P;
      if (2 * P <= ny) launch_row<T, N, MODE, true, RC::vpt, RC::split, RC::pairs>(nlines / 2, ny, psi, pc, scale, tw, s, st);
      else launch_row<T, N, MODE, false, RC::vpt, RC::split, RC::pairs>(nlines / 2, ny, psi, pc, scale, tw, s, st);
      ok = true;
    };
    if (mode == 0) {
      pairs(IntC<0>{}, RowCfg<C::VPT, C::SPLIT, line_radix(N), 0>{});
    } else if (mode == 2) {
      pairs(IntC<2>{}, RowCfg<C::VPT, C::SPLIT, line_radix(N), 0>{});
    } else {
      dispatch_nls_row<T, N>(var, [&](auto cfg) {
        using RC = decltype(cfg);
        if constexpr (NlsRowShape<N>::ONE_LINE) {
          // one line per block, mapped so that each XCD takes a contiguous
          // range of lines (the two lines of a pair share its L2)
          auto* k = &k_nls_row1<T, N, 1, RC::vpt, RC::split, RC::radix>;
          constexpr size_t lds = (size_t)lds_line_len(N) * (RC::split ? sizeof(T) : sizeof(cpx<T>));
          allow_lds(k, lds);
          hipLaunchKernelGGL(k, dim3(nlines), dim3(N / RC::vpt), lds, s, psi, ilog2c(ny), (T)pc, (T)scale,
                             (const cpx<T>*)tw);
          ok = true;
        } else {
          pairs(IntC<1>{}, cfg);
        }
      });
    }
  });
  return ok ? hipGetLastError() : hipErrorInvalidValue;
}

hipError_t nls_row(Prec p, int nx, int nlines, int ny, FieldRef psi, int mode, double phase_coef, double scale,
                   const void* tw, hipStream_t s, StatusRef st, int var) {
  return p == P32 ? row<float>(nx, nlines, ny, psi, mode, phase_coef, scale, tw, s, st, var)
                  : row<double>(nx, nlines, ny, psi, mode, phase_coef, scale, tw, s, st, var);
}

bool nls_row_variant_info(Prec p, int n, int var, int* pairs, int* vpt, int* split, int* radix) {
  bool found = false;
  dispatch_n(n, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    auto get = [&](auto cfg) {
      using RC = decltype(cfg);
      // pairs: row pairs per block, 0 for one line per block
      *pairs = NlsRowShape<N>::ONE_LINE ? 0 : PairGeom<float, N, RC::vpt, RC::split, RC::pairs>::P;
      *vpt = RC::vpt;
      *split = RC::split ? 1 : 0;
      *radix = RC::radix;
      found = true;
    };
    if (p == P32) dispatch_nls_row<float, N>(var, get);
    else dispatch_nls_row<double, N>(var, get);
  });
  return found;
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
      auto* k = &k_nls_col<T, N, C::w, C::vpt, C::split, C::wpe, C::radix>;
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
