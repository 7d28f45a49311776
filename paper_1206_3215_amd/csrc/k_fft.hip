// Plain 2D transform passes: complex rows, complex columns, and pairs of
// real rows (real-to-half-spectrum and back).
#include "kernels.hpp"
#include "launch.hpp"

namespace pst {

// ------------------------------------------------------------ C2C rows ---
template <typename T, int N, bool INV>
__global__ __launch_bounds__((RowGeom<T, N>::THREADS)) void k_row_c2c(
    const cpx<T>* in, cpx<T>* out, int nlines, T scale, const cpx<T>* __restrict__ tw) {
  using G = RowGeom<T, N>;
  extern __shared__ char smem[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem);
  const int lid = threadIdx.x / G::TL, t = threadIdx.x % G::TL;
  const int line = blockIdx.x * G::LPB + lid;
  const bool valid = line < nlines;
  cpx<T>* L = lds + lid * lds_line_stride<T>(N);
  cpx<T> v[G::R];
  const cpx<T>* src = in + (size_t)line * N;
#pragma unroll
  for (int s = 0; s < G::R; ++s) v[s] = valid ? src[t + s * G::TL] : cpx<T>{0, 0};
  line_fft<N, INV>(v, L, t, tw);
  if (valid) {
    cpx<T>* dst = out + (size_t)line * N;
#pragma unroll
    for (int s = 0; s < G::R; ++s) gstore(dst + (t + s * G::TL), v[s] * scale);
  }
}

// --------------------------------------------------------- C2C columns ---
template <typename T, int N, bool INV, int WT, int VPT, bool SPLIT, int WPE, int R>
__global__ __launch_bounds__((WT * (N / VPT))) __attribute__((amdgpu_waves_per_eu(WPE))) void k_col_c2c(
    const cpx<T>* src, cpx<T>* dst, int ncols, int ld, int tiles_per_field, T scale, const cpx<T>* __restrict__ tw) {
  using G = ColGeom<T, N, WT, VPT, SPLIT>;
  extern __shared__ char smem[];
  const int c = threadIdx.x % WT, t = threadIdx.x / WT;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int fld = tile / tiles_per_field;
  const int col = (tile % tiles_per_field) * WT + c;
  const bool valid = col < ncols;
  const int cc = valid ? col : ncols - 1;  // columns past the end recompute the last one, unstored
  const size_t fbytes = (size_t)N * ld * sizeof(cpx<T>);
  const FieldBuf in((const char*)src + fld * fbytes, (unsigned)fbytes);
  const FieldBuf out((char*)dst + fld * fbytes, (unsigned)fbytes);
  const unsigned o0 = (unsigned)(cc + t * ld) * (unsigned)sizeof(cpx<T>);
  const unsigned ds = (unsigned)(G::TL * ld) * (unsigned)sizeof(cpx<T>);
  void* L = SPLIT ? (void*)(reinterpret_cast<T*>(smem) + c) : (void*)(reinterpret_cast<cpx<T>*>(smem) + c);
  cpx<T> v[G::R];
#pragma unroll
  for (int s = 0; s < G::R; ++s) v[s] = in.template ldc<T>(o0, s * ds);
  line_fft<N, INV, WT, VPT, SPLIT, R>(v, L, t, tw);
  if (valid) {
#pragma unroll
    for (int s = 0; s < G::R; ++s) out.st(o0, s * ds, v[s] * scale);
  }
}

// ----------------------------------------------------- real row pairs ---
// Rows 2p and 2p+1 travel as one complex line z = a + i b.
template <typename T, int N>
__global__ __launch_bounds__((RowGeom<T, N>::THREADS)) void k_row_r2c(
    FieldRef in, cpx<T>* out, int nlines, int lny, const cpx<T>* __restrict__ tw) {
  using G = RowGeom<T, N>;
  constexpr int H = N / 2 + 1;
  extern __shared__ char smem[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem);
  const int lid = threadIdx.x / G::TL, t = threadIdx.x % G::TL;
  const int pair = blockIdx.x * G::LPB + lid;
  const int la = 2 * pair, lb = 2 * pair + 1;
  const bool va = la < nlines, vb = lb < nlines;
  cpx<T>* L = lds + lid * lds_line_stride<T>(N);
  cpx<T> v[G::R];
  const int ny = 1 << lny;
  gptr<const T> ra = field<const T>(in, la >> lny) + (size_t)(la & (ny - 1)) * N;
  gptr<const T> rb = ra + N;
#pragma unroll
  for (int s = 0; s < G::R; ++s) {
    const int e = t + s * G::TL;
    v[s] = cpx<T>{va ? ra[e] : T(0), vb ? rb[e] : T(0)};
  }
  line_fft<N, false>(v, L, t, tw);
#pragma unroll
  for (int s = 0; s < G::R; ++s) L[lds_idx(t + s * G::TL)] = v[s];
  __syncthreads();
  cpx<T>* oa = out + (size_t)la * H;
  cpx<T>* ob = out + (size_t)lb * H;
#pragma unroll
  for (int s = 0; s <= G::R / 2; ++s) {
    const int k = (s < G::R / 2) ? t + s * G::TL : N / 2;
    if (s == G::R / 2 && t != 0) break;
    const cpx<T> zk = L[lds_idx(k)];
    const cpx<T> zm = conj(L[lds_idx((N - k) & (N - 1))]);
    const cpx<T> sum = zk + zm, dif = zk - zm;
    if (va) gstore(oa + k, sum * T(0.5));
    if (vb) gstore(ob + k, cpx<T>{dif.im, -dif.re} * T(0.5));
  }
}

template <typename T, int N>
__global__ __launch_bounds__((RowGeom<T, N>::THREADS)) void k_row_c2r(
    const cpx<T>* in, FieldRef out, int nlines, int lny, T scale, const cpx<T>* __restrict__ tw, const int* skip) {
  using G = RowGeom<T, N>;
  constexpr int H = N / 2 + 1;
  extern __shared__ char smem[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem);
  const int lid = threadIdx.x / G::TL, t = threadIdx.x % G::TL;
  const int pair = blockIdx.x * G::LPB + lid;
  const int la = 2 * pair, lb = 2 * pair + 1;
  const bool va = la < nlines, vb = lb < nlines;
  cpx<T>* L = lds + lid * lds_line_stride<T>(N);
  const cpx<T>* xa = in + (size_t)la * H;
  const cpx<T>* xb = in + (size_t)lb * H;
  cpx<T> v[G::R];
#pragma unroll
  for (int s = 0; s < G::R; ++s) {
    const int e = t + s * G::TL;
    const bool lo = e <= N / 2;
    const int k = lo ? e : N - e;
    cpx<T> A = va ? xa[k] : cpx<T>{0, 0};
    cpx<T> B = vb ? xb[k] : cpx<T>{0, 0};
    if (e == 0 || e == N / 2) {
      A.im = 0;
      B.im = 0;
    }
    if (!lo) {
      A = conj(A);
      B = conj(B);
    }
    v[s] = A + mul_i(B);
  }
  line_fft<N, true>(v, L, t, tw);
  const int ny = 1 << lny;
  // (rows a and b lie in one field: ny is even)
  if (skip != nullptr && va && skip[la >> lny]) return;
  gptr<T> oa = field<T>(out, la >> lny) + (size_t)(la & (ny - 1)) * N;
  gptr<T> ob = oa + N;
#pragma unroll
  for (int s = 0; s < G::R; ++s) {
    const int e = t + s * G::TL;
    if (va) oa[e] = v[s].re * scale;
    if (vb) ob[e] = v[s].im * scale;
  }
}

// ----------------------------------------------------------- launchers ---
template <typename T>
static hipError_t row_c2c(int n, int nlines, const void* in, void* out, bool inv, double scale,
                          const void* tw, hipStream_t s) {
  bool ok = dispatch_n(n, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    using G = RowGeom<T, N>;
    const int grid = (nlines + G::LPB - 1) / G::LPB;
    if (inv) {
      allow_lds((k_row_c2c<T, N, true>), G::LDS_BYTES);
      hipLaunchKernelGGL((k_row_c2c<T, N, true>), dim3(grid), dim3(G::THREADS), G::LDS_BYTES, s,
                         (const cpx<T>*)in, (cpx<T>*)out, nlines, (T)scale, (const cpx<T>*)tw);
    } else {
      allow_lds((k_row_c2c<T, N, false>), G::LDS_BYTES);
      hipLaunchKernelGGL((k_row_c2c<T, N, false>), dim3(grid), dim3(G::THREADS), G::LDS_BYTES, s,
                         (const cpx<T>*)in, (cpx<T>*)out, nlines, (T)scale, (const cpx<T>*)tw);
    }
  });
  return ok ? hipGetLastError() : hipErrorInvalidValue;
}

hipError_t fft_row_c2c(Prec p, int n, int nlines, const void* in, void* out, bool inv, double scale,
                       const void* tw, hipStream_t s) {
  return p == P32 ? row_c2c<float>(n, nlines, in, out, inv, scale, tw, s)
                  : row_c2c<double>(n, nlines, in, out, inv, scale, tw, s);
}

template <typename T>
static hipError_t col_c2c(int ny, int ncols, int ld, int nfields, const void* src, void* dst, bool inv,
                          double scale, const void* tw, int W, hipStream_t s) {
  bool ok = false;
  dispatch_n(ny, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    ok = dispatch_col1<T, N>(W, [&](auto cfg) {
      using C = decltype(cfg);
      using G = ColGeom<T, N, C::w, C::vpt, C::split>;
      const int tiles = (ncols + C::w - 1) / C::w;
      auto* k = inv ? &k_col_c2c<T, N, true, C::w, C::vpt, C::split, C::wpe, C::radix>
                    : &k_col_c2c<T, N, false, C::w, C::vpt, C::split, C::wpe, C::radix>;
      allow_lds(k, G::LDS_BYTES);
      hipLaunchKernelGGL(k, dim3(tiles * nfields), dim3(G::THREADS), G::LDS_BYTES, s, (const cpx<T>*)src,
                         (cpx<T>*)dst, ncols, ld, tiles, (T)scale, (const cpx<T>*)tw);
    });
  });
  return ok ? hipGetLastError() : hipErrorInvalidValue;
}

hipError_t fft_col_c2c(Prec p, int ny, int ncols, int ld, int nfields, const void* src, void* dst,
                       bool inv, double scale, const void* tw, int W, hipStream_t s) {
  return p == P32 ? col_c2c<float>(ny, ncols, ld, nfields, src, dst, inv, scale, tw, W, s)
                  : col_c2c<double>(ny, ncols, ld, nfields, src, dst, inv, scale, tw, W, s);
}

template <typename T>
static hipError_t row_r2c(int n, int nlines, int ny, FieldRef in, void* out, const void* tw,
                          hipStream_t s) {
  bool ok = dispatch_n(n, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    using G = RowGeom<T, N>;
    const int pairs = (nlines + 1) / 2;
    const int grid = (pairs + G::LPB - 1) / G::LPB;
    allow_lds((k_row_r2c<T, N>), G::LDS_BYTES);
    hipLaunchKernelGGL((k_row_r2c<T, N>), dim3(grid), dim3(G::THREADS), G::LDS_BYTES, s,
                       in, (cpx<T>*)out, nlines, ilog2c(ny), (const cpx<T>*)tw);
  });
  return ok ? hipGetLastError() : hipErrorInvalidValue;
}

hipError_t fft_row_r2c(Prec p, int n, int nlines, int ny, FieldRef in, void* out, const void* tw,
                       hipStream_t s) {
  return p == P32 ? row_r2c<float>(n, nlines, ny, in, out, tw, s) : row_r2c<double>(n, nlines, ny, in, out, tw, s);
}

template <typename T>
static hipError_t row_c2r(int n, int nlines, int ny, const void* in, FieldRef out, double scale,
                          const void* tw, hipStream_t s, const int* skip) {
  bool ok = dispatch_n(n, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    using G = RowGeom<T, N>;
    const int pairs = (nlines + 1) / 2;
    const int grid = (pairs + G::LPB - 1) / G::LPB;
    allow_lds((k_row_c2r<T, N>), G::LDS_BYTES);
    hipLaunchKernelGGL((k_row_c2r<T, N>), dim3(grid), dim3(G::THREADS), G::LDS_BYTES, s,
                       (const cpx<T>*)in, out, nlines, ilog2c(ny), (T)scale, (const cpx<T>*)tw, skip);
  });
  return ok ? hipGetLastError() : hipErrorInvalidValue;
}

hipError_t fft_row_c2r(Prec p, int n, int nlines, int ny, const void* in, FieldRef out, double scale,
                       const void* tw, hipStream_t s, const int* skip) {
  return p == P32 ? row_c2r<float>(n, nlines, ny, in, out, scale, tw, s, skip)
                  : row_c2r<double>(n, nlines, ny, in, out, scale, tw, s, skip);
}

bool col_variant_info(Prec p, int n, int var, bool single, int* w, int* vpt, int* split, int* radix) {
  bool found = false;
  auto get = [&](auto cfg) {
    using C = decltype(cfg);
    *w = C::w;
    *vpt = C::vpt;
    *split = C::split ? 1 : 0;
    *radix = C::radix;
    found = true;
  };
  dispatch_n(n, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    if (single) {
      if (p == P32) dispatch_col1<float, N>(var, get);
      else dispatch_col1<double, N>(var, get);
    } else {
      auto getw = [&](auto wc) { get(ColCfg<decltype(wc)::value, line_radix(N), false, 1, line_radix(N)>{}); };
      if (p == P32) dispatch_w<float, N>(var, getw);
      else dispatch_w<double, N>(var, getw);
    }
  });
  return found;
}

}  // namespace pst
