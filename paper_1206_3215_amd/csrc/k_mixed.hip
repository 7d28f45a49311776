// Mixed-radix passes for line lengths n = 2^a 3^b 5^c that are not powers
// of two (the register-resident Stockham kernels need the values a thread
// holds to be a multiple of every stage radix, which mixed radices break).
//
// A block transforms W lines held in LDS, interleaved (element e of line c
// at e*W + c), in two buffers it alternates between: every stage reads one
// and writes the other, so a thread needs the values of one butterfly at a
// time and the stage list can be a runtime table.  A stage of radix r
// (2, 3, 4, 5 or 8) with Ns = product of the earlier radices runs the n/r
// butterflies j: inputs src[j + q n/r], twiddles exp(-+2 pi i q k/(Ns r))
// with k = j mod Ns from the length's table ((r-1) Ns entries per stage,
// computed in double precision on the host and rounded once), outputs to
// dst[(j/Ns) Ns r + k + q Ns] (Stockham autosort: natural order at the end).
//
// The NLS passes keep the hybrid field (transformed along x only) in plain
// row order; the two-line pair layout of the power-of-two passes is not
// used here.  The phase and propagator arithmetic is that of k_nls.hip.
#include "kernels.hpp"
#include "launch.hpp"

namespace pst {

namespace {

constexpr int kMxThreads = 256;

// DFT of length 3 in place (forward kernel exp(-2 pi i/3); INV: conjugate).
template <bool INV, typename T>
__device__ __forceinline__ void dft3(cpx<T>* x) {
  const T h = T(0.86602540378443864676);  // sin(2 pi/3)
  const cpx<T> s = x[1] + x[2], d = x[1] - x[2];
  const cpx<T> m = cpx<T>{x[0].re - T(0.5) * s.re, x[0].im - T(0.5) * s.im};
  // -i h d (forward) or +i h d (inverse)
  const cpx<T> r = INV ? cpx<T>{-h * d.im, h * d.re} : cpx<T>{h * d.im, -h * d.re};
  x[0] = x[0] + s;
  x[1] = m + r;
  x[2] = m - r;
}

// DFT of length 5 in place, from the sums and differences of the
// conjugate-symmetric input pairs (1, 4) and (2, 3).
template <bool INV, typename T>
__device__ __forceinline__ void dft5(cpx<T>* x) {
  const T c1 = T(0.30901699437494742410), c2 = T(-0.80901699437494742410);  // cos(2 pi/5), cos(4 pi/5)
  const T s1 = T(0.95105651629515357212), s2 = T(0.58778525229247312917);   // sin(2 pi/5), sin(4 pi/5)
  const cpx<T> a1 = x[1] + x[4], a2 = x[2] + x[3], b1 = x[1] - x[4], b2 = x[2] - x[3];
  const cpx<T> p1 = cpx<T>{x[0].re + c1 * a1.re + c2 * a2.re, x[0].im + c1 * a1.im + c2 * a2.im};
  const cpx<T> p2 = cpx<T>{x[0].re + c2 * a1.re + c1 * a2.re, x[0].im + c2 * a1.im + c1 * a2.im};
  const cpx<T> q1 = cpx<T>{s1 * b1.re + s2 * b2.re, s1 * b1.im + s2 * b2.im};
  const cpx<T> q2 = cpx<T>{s2 * b1.re - s1 * b2.re, s2 * b1.im - s1 * b2.im};
  // -i q (forward) or +i q (inverse)
  const cpx<T> r1 = INV ? cpx<T>{-q1.im, q1.re} : cpx<T>{q1.im, -q1.re};
  const cpx<T> r2 = INV ? cpx<T>{-q2.im, q2.re} : cpx<T>{q2.im, -q2.re};
  x[0] = x[0] + a1 + a2;
  x[1] = p1 + r1;
  x[4] = p1 - r1;
  x[2] = p2 + r2;
  x[3] = p2 - r2;
}

template <int R, bool INV, typename T>
__device__ __forceinline__ void dft_r(cpx<T>* x) {
  if constexpr (R == 2) dft2<INV>(x[0], x[1]);
  else if constexpr (R == 3) dft3<INV>(x);
  else if constexpr (R == 4) dft4<INV>(x[0], x[1], x[2], x[3]);
  else if constexpr (R == 5) dft5<INV>(x);
  else dft8<INV>(x);
}

// Butterfly j of a stage of radix R.
template <int R, bool INV, typename T>
__device__ __forceinline__ void mx_bfly(const cpx<T>* src, cpx<T>* dst, int W, int c, int j, int n, int Ns,
                                        const cpx<T>* __restrict__ tw, int toff) {
  const int m = n / R, k = j % Ns;
  cpx<T> x[R];
#pragma unroll
  for (int q = 0; q < R; ++q) x[q] = src[(j + q * m) * W + c];
  if (Ns > 1) {
#pragma unroll
    for (int q = 1; q < R; ++q) {
      const cpx<T> w = tw[toff + (q - 1) * Ns + k];
      x[q] = INV ? cmul_conj(x[q], w) : cmul(x[q], w);
    }
  }
  dft_r<R, INV>(x);
  const int base = (j / Ns) * Ns * R + k;
#pragma unroll
  for (int q = 0; q < R; ++q) dst[(base + q * Ns) * W + c] = x[q];
}

// Transform the W lines held in A (interleaved); every thread of the block
// calls it.  Returns the buffer (A or B) that holds the result.
template <bool INV, typename T>
__device__ cpx<T>* mx_fft(cpx<T>* A, cpx<T>* B, int W, const MixedLine& ml, const cpx<T>* __restrict__ tw) {
  const int c = threadIdx.x % W, lt = threadIdx.x / W, nth = blockDim.x / W;
  cpx<T>* src = A;
  cpx<T>* dst = B;
  for (int s = 0; s < ml.nst; ++s) {
    const int r = ml.r[s], Ns = ml.ns[s], toff = ml.toff[s], m = ml.n / r;
    for (int j = lt; j < m; j += nth) {
      switch (r) {
        case 2: mx_bfly<2, INV>(src, dst, W, c, j, ml.n, Ns, tw, toff); break;
        case 3: mx_bfly<3, INV>(src, dst, W, c, j, ml.n, Ns, tw, toff); break;
        case 4: mx_bfly<4, INV>(src, dst, W, c, j, ml.n, Ns, tw, toff); break;
        case 5: mx_bfly<5, INV>(src, dst, W, c, j, ml.n, Ns, tw, toff); break;
        default: mx_bfly<8, INV>(src, dst, W, c, j, ml.n, Ns, tw, toff); break;
      }
    }
    __syncthreads();
    cpx<T>* t = src;
    src = dst;
    dst = t;
  }
  return src;
}

// ------------------------------------------------------------- C2C passes ---
// Rows: W lines per block, each contiguous.
template <typename T, bool INV>
__global__ __launch_bounds__(kMxThreads) void k_mx_row_c2c(const cpx<T>* in, cpx<T>* out, int nlines, int W, T scale,
                                                           MixedLine ml, const cpx<T>* __restrict__ tw) {
  extern __shared__ char smem[];
  const int n = ml.n;
  cpx<T>* A = reinterpret_cast<cpx<T>*>(smem);
  cpx<T>* B = A + (size_t)W * n;
  const int l0 = blockIdx.x * W;
  for (int i = threadIdx.x; i < W * n; i += blockDim.x) {
    const int c = i / n, e = i % n;
    A[e * W + c] = l0 + c < nlines ? in[(size_t)(l0 + c) * n + e] : cpx<T>{0, 0};
  }
  __syncthreads();
  const cpx<T>* res = mx_fft<INV>(A, B, W, ml, tw);
  for (int i = threadIdx.x; i < W * n; i += blockDim.x) {
    const int c = i / n, e = i % n;
    if (l0 + c < nlines) gstore(out + ((size_t)(l0 + c) * n + e), res[e * W + c] * scale);
  }
}

// Columns: W adjacent columns of a field per block ([field][n][ld] layout,
// the first ncols columns of each row transformed).
template <typename T, bool INV>
__global__ __launch_bounds__(kMxThreads) void k_mx_col_c2c(const cpx<T>* src, cpx<T>* dst, int ncols, int ld,
                                                           int tiles_per_field, int W, T scale, MixedLine ml,
                                                           const cpx<T>* __restrict__ tw) {
  extern __shared__ char smem[];
  const int n = ml.n;
  cpx<T>* A = reinterpret_cast<cpx<T>*>(smem);
  cpx<T>* B = A + (size_t)W * n;
  const int field = blockIdx.x / tiles_per_field, col0 = (blockIdx.x % tiles_per_field) * W;
  const size_t fo = (size_t)field * n * ld;
  for (int i = threadIdx.x; i < W * n; i += blockDim.x) {
    const int e = i / W, c = i % W;
    A[e * W + c] = col0 + c < ncols ? src[fo + (size_t)e * ld + col0 + c] : cpx<T>{0, 0};
  }
  __syncthreads();
  const cpx<T>* res = mx_fft<INV>(A, B, W, ml, tw);
  for (int i = threadIdx.x; i < W * n; i += blockDim.x) {
    const int e = i / W, c = i % W;
    if (col0 + c < ncols) gstore(dst + (fo + (size_t)e * ld + col0 + c), res[e * W + c] * scale);
  }
}

// ------------------------------------------------------------ real rows ---
// R2C: each real row as a complex line (imaginary part 0), first n/2+1
// outputs kept.  C2R: the full spectrum rebuilt from the half by Hermitian
// symmetry (imaginary parts of the self-conjugate modes dropped), real part
// of the inverse kept, times scale.
template <typename T>
__global__ __launch_bounds__(kMxThreads) void k_mx_row_r2c(const T* in, cpx<T>* out, int nlines, int W, MixedLine ml,
                                                           const cpx<T>* __restrict__ tw) {
  extern __shared__ char smem[];
  const int n = ml.n, h = n / 2 + 1;
  cpx<T>* A = reinterpret_cast<cpx<T>*>(smem);
  cpx<T>* B = A + (size_t)W * n;
  const int l0 = blockIdx.x * W;
  for (int i = threadIdx.x; i < W * n; i += blockDim.x) {
    const int c = i / n, e = i % n;
    A[e * W + c] = cpx<T>{l0 + c < nlines ? in[(size_t)(l0 + c) * n + e] : T(0), T(0)};
  }
  __syncthreads();
  const cpx<T>* res = mx_fft<false>(A, B, W, ml, tw);
  for (int i = threadIdx.x; i < W * h; i += blockDim.x) {
    const int c = i / h, e = i % h;
    if (l0 + c < nlines) gstore(out + ((size_t)(l0 + c) * h + e), res[e * W + c]);
  }
}

template <typename T>
__global__ __launch_bounds__(kMxThreads) void k_mx_row_c2r(const cpx<T>* in, T* out, int nlines, int W, T scale,
                                                           MixedLine ml, const cpx<T>* __restrict__ tw) {
  extern __shared__ char smem[];
  const int n = ml.n, h = n / 2 + 1;
  cpx<T>* A = reinterpret_cast<cpx<T>*>(smem);
  cpx<T>* B = A + (size_t)W * n;
  const int l0 = blockIdx.x * W;
  for (int i = threadIdx.x; i < W * n; i += blockDim.x) {
    const int c = i / n, e = i % n;
    cpx<T> x{0, 0};
    if (l0 + c < nlines) {
      const cpx<T>* row = in + (size_t)(l0 + c) * h;
      if (e < h) {
        x = row[e];
        if (e == 0 || 2 * e == n) x.im = 0;
      } else {
        x = conj(row[n - e]);
      }
    }
    A[e * W + c] = x;
  }
  __syncthreads();
  const cpx<T>* res = mx_fft<true>(A, B, W, ml, tw);
  for (int i = threadIdx.x; i < W * n; i += blockDim.x) {
    const int c = i / n, e = i % n;
    if (l0 + c < nlines) store1(out + ((size_t)(l0 + c) * n + e), res[e * W + c].re * scale);
  }
}

// ------------------------------------------------------------------ NLS ---
// Row pass, modes as nls_row: 0 H = scale FFT_x(psi); 1 H <- FFT_x(e^{-i c
// |iFFT_x H|^2} iFFT_x H); 2 psi = scale iFFT_x(H), latching a non-finite
// field into st.  Lines are rows of fields of ny rows (a field per line).
template <typename T, int MODE>
__global__ __launch_bounds__(kMxThreads) void k_mx_nls_row(FieldRef psi, int nlines, int ny, int W, T phase_coef,
                                                           T scale, MixedLine ml, const cpx<T>* __restrict__ tw,
                                                           StatusRef st) {
  extern __shared__ char smem[];
  const int n = ml.n;
  cpx<T>* A = reinterpret_cast<cpx<T>*>(smem);
  cpx<T>* B = A + (size_t)W * n;
  const int l0 = blockIdx.x * W;
  auto row = [&](int line) { return reinterpret_cast<cpx<T>*>(psi.at(line / ny)) + (size_t)(line % ny) * n; };
  for (int i = threadIdx.x; i < W * n; i += blockDim.x) {
    const int c = i / n, e = i % n;
    A[e * W + c] = l0 + c < nlines ? row(l0 + c)[e] : cpx<T>{0, 0};
  }
  __syncthreads();
  cpx<T>* res;
  if constexpr (MODE == 0) {
    res = mx_fft<false>(A, B, W, ml, tw);
  } else if constexpr (MODE == 1) {
    res = mx_fft<true>(A, B, W, ml, tw);
    for (int i = threadIdx.x; i < W * n; i += blockDim.x) res[i] = rotate_neg(res[i], phase_coef * norm2(res[i]));
    __syncthreads();
    res = mx_fft<false>(res, res == A ? B : A, W, ml, tw);
  } else {
    res = mx_fft<true>(A, B, W, ml, tw);
  }
  bool bad = false;
  for (int i = threadIdx.x; i < W * n; i += blockDim.x) {
    const int c = i / n, e = i % n;
    if (l0 + c < nlines) {
      const cpx<T> v = MODE == 1 ? res[e * W + c] : res[e * W + c] * scale;
      gstore(row(l0 + c) + e, v);
      if constexpr (MODE == 2) bad = bad || !finite_c(v);
    }
  }
  if constexpr (MODE == 2) {
    // a thread's elements may belong to several fields: latch each line's own
    for (int i = threadIdx.x; bad && i < W * n; i += blockDim.x) {
      const int c = i / n, e = i % n;
      if (l0 + c < nlines && !finite_c(res[e * W + c])) latch_nonfinite(true, st, (l0 + c) / ny, false);
    }
  }
}

// Column pass: FFT_y, multiply by (1 + ex[mx]) (1 + ey[my]) scale, iFFT_y.
template <typename T>
__global__ __launch_bounds__(kMxThreads) void k_mx_nls_col(FieldRef psi, int nx, int tiles_per_field, int W, T scale,
                                                           MixedLine ml, const cpx<T>* __restrict__ tw,
                                                           const cpx<T>* __restrict__ ex,
                                                           const cpx<T>* __restrict__ ey) {
  extern __shared__ char smem[];
  const int n = ml.n;
  cpx<T>* A = reinterpret_cast<cpx<T>*>(smem);
  cpx<T>* B = A + (size_t)W * n;
  const int field = blockIdx.x / tiles_per_field, col0 = (blockIdx.x % tiles_per_field) * W;
  cpx<T>* f = reinterpret_cast<cpx<T>*>(psi.at(field));
  for (int i = threadIdx.x; i < W * n; i += blockDim.x) {
    const int e = i / W, c = i % W;
    A[e * W + c] = col0 + c < nx ? f[(size_t)e * nx + col0 + c] : cpx<T>{0, 0};
  }
  __syncthreads();
  cpx<T>* res = mx_fft<false>(A, B, W, ml, tw);
  for (int i = threadIdx.x; i < W * n; i += blockDim.x) {
    const int e = i / W, c = i % W;
    const int cc = col0 + c < nx ? col0 + c : nx - 1;
    const cpx<T> w = res[i] * scale;
    const cpx<T> wx = w + cmul(w, ex[cc]);
    res[i] = wx + cmul(wx, ey[e]);
  }
  __syncthreads();
  const cpx<T>* out = mx_fft<true>(res, res == A ? B : A, W, ml, tw);
  for (int i = threadIdx.x; i < W * n; i += blockDim.x) {
    const int e = i / W, c = i % W;
    if (col0 + c < nx) gstore(f + ((size_t)e * nx + col0 + c), out[i]);
  }
}

// NLS diagnostics: line sums of |psi|^2 and |psi|^4 into part[2 line + {0,1}]
// with spec = FFT_x(psi); then FFT_y of spec and column sums of
// |k|^2 |psi_hat|^2 into part[field nx + col].  Double accumulation, fixed
// order (strided per thread, then a fixed tree over the block's threads).
template <typename T>
__global__ __launch_bounds__(kMxThreads) void k_mx_cq_row(const cpx<T>* psi, cpx<T>* spec, int nlines, double* part,
                                                          MixedLine ml, const cpx<T>* __restrict__ tw) {
  extern __shared__ char smem[];
  __shared__ double red[kMxThreads];
  const int n = ml.n, line = blockIdx.x;
  cpx<T>* A = reinterpret_cast<cpx<T>*>(smem);
  cpx<T>* B = A + n;
  double m2 = 0.0, m4 = 0.0;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const cpx<T> v = psi[(size_t)line * n + e];
    A[e] = v;
    const double a = (double)v.re * v.re + (double)v.im * v.im;
    m2 += a;
    m4 += a * a;
  }
  m2 = line_sum(red, 0, threadIdx.x, kMxThreads, m2);
  m4 = line_sum(red, 0, threadIdx.x, kMxThreads, m4);
  if (threadIdx.x == 0) {
    store1(part + 2 * (size_t)line, m2);
    store1(part + 2 * (size_t)line + 1, m4);
  }
  const cpx<T>* res = mx_fft<false>(A, B, 1, ml, tw);
  for (int e = threadIdx.x; e < n; e += blockDim.x) gstore(spec + ((size_t)line * n + e), res[e]);
}

template <typename T>
__global__ __launch_bounds__(kMxThreads) void k_mx_cq_col(const cpx<T>* spec, int nx, double* part, MixedLine ml,
                                                          const cpx<T>* __restrict__ tw, double kx0, double ky0) {
  extern __shared__ char smem[];
  __shared__ double red[kMxThreads];
  const int n = ml.n, field = blockIdx.x / nx, col = blockIdx.x % nx;
  cpx<T>* A = reinterpret_cast<cpx<T>*>(smem);
  cpx<T>* B = A + n;
  for (int e = threadIdx.x; e < n; e += blockDim.x) A[e] = spec[((size_t)field * n + e) * nx + col];
  __syncthreads();
  const cpx<T>* res = mx_fft<false>(A, B, 1, ml, tw);
  const int mx = col < (nx + 1) / 2 ? col : col - nx;
  const double kx = kx0 * mx;
  double acc = 0.0;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int my = e < (n + 1) / 2 ? e : e - n;
    const double ky = ky0 * my;
    acc += (kx * kx + ky * ky) * ((double)res[e].re * res[e].re + (double)res[e].im * res[e].im);
  }
  acc = line_sum(red, 0, threadIdx.x, kMxThreads, acc);
  if (threadIdx.x == 0) part[(size_t)field * nx + col] = acc;
}

// Lines per block: as many as fit 150 KB of LDS (two buffers), at most 16,
// and no more than the block's threads can share (16 threads per line).
template <typename T>
int lines_per_block(int n) {
  int w = 16;
  while (w > 1 && (2 * (size_t)w * n * sizeof(cpx<T>) > 150 * 1024 || w * n > 64 * kMxThreads)) w /= 2;
  return w;
}

template <typename T>
size_t lds_bytes(int w, int n) {
  return 2 * (size_t)w * n * sizeof(cpx<T>);
}

template <class K>
void allow(K k, size_t bytes) {
  allow_lds(k, bytes);
}

}  // namespace

bool mixed_supported(Prec p, int n) {
  return 2 * (size_t)n * (p == P32 ? sizeof(cpx<float>) : sizeof(cpx<double>)) <= 150 * 1024;
}

template <typename T>
static hipError_t mx_row_c2c(const MixedLine& ml, int nlines, const void* in, void* out, bool inv, double scale,
                             const void* tw, hipStream_t s) {
  const int W = lines_per_block<T>(ml.n);
  const size_t lds = lds_bytes<T>(W, ml.n);
  const dim3 grid((nlines + W - 1) / W);
  if (inv) {
    allow(k_mx_row_c2c<T, true>, lds);
    hipLaunchKernelGGL((k_mx_row_c2c<T, true>), grid, dim3(kMxThreads), lds, s, (const cpx<T>*)in, (cpx<T>*)out,
                       nlines, W, (T)scale, ml, (const cpx<T>*)tw);
  } else {
    allow(k_mx_row_c2c<T, false>, lds);
    hipLaunchKernelGGL((k_mx_row_c2c<T, false>), grid, dim3(kMxThreads), lds, s, (const cpx<T>*)in, (cpx<T>*)out,
                       nlines, W, (T)scale, ml, (const cpx<T>*)tw);
  }
  return hipGetLastError();
}

hipError_t mixed_row_c2c(Prec p, const MixedLine& ml, int nlines, const void* in, void* out, bool inv, double scale,
                         const void* tw, hipStream_t s) {
  return p == P32 ? mx_row_c2c<float>(ml, nlines, in, out, inv, scale, tw, s)
                  : mx_row_c2c<double>(ml, nlines, in, out, inv, scale, tw, s);
}

template <typename T>
static hipError_t mx_col_c2c(const MixedLine& ml, int ncols, int ld, int nfields, const void* src, void* dst, bool inv,
                             double scale, const void* tw, hipStream_t s) {
  const int W = lines_per_block<T>(ml.n);
  const size_t lds = lds_bytes<T>(W, ml.n);
  const int tiles = (ncols + W - 1) / W;
  if (inv) {
    allow(k_mx_col_c2c<T, true>, lds);
    hipLaunchKernelGGL((k_mx_col_c2c<T, true>), dim3(tiles * nfields), dim3(kMxThreads), lds, s, (const cpx<T>*)src,
                       (cpx<T>*)dst, ncols, ld, tiles, W, (T)scale, ml, (const cpx<T>*)tw);
  } else {
    allow(k_mx_col_c2c<T, false>, lds);
    hipLaunchKernelGGL((k_mx_col_c2c<T, false>), dim3(tiles * nfields), dim3(kMxThreads), lds, s, (const cpx<T>*)src,
                       (cpx<T>*)dst, ncols, ld, tiles, W, (T)scale, ml, (const cpx<T>*)tw);
  }
  return hipGetLastError();
}

hipError_t mixed_col_c2c(Prec p, const MixedLine& ml, int ncols, int ld, int nfields, const void* src, void* dst,
                         bool inv, double scale, const void* tw, hipStream_t s) {
  return p == P32 ? mx_col_c2c<float>(ml, ncols, ld, nfields, src, dst, inv, scale, tw, s)
                  : mx_col_c2c<double>(ml, ncols, ld, nfields, src, dst, inv, scale, tw, s);
}

template <typename T>
static hipError_t mx_row_r2c(const MixedLine& ml, int nlines, const void* in, void* out, const void* tw,
                             hipStream_t s) {
  const int W = lines_per_block<T>(ml.n);
  const size_t lds = lds_bytes<T>(W, ml.n);
  allow(k_mx_row_r2c<T>, lds);
  hipLaunchKernelGGL((k_mx_row_r2c<T>), dim3((nlines + W - 1) / W), dim3(kMxThreads), lds, s, (const T*)in,
                     (cpx<T>*)out, nlines, W, ml, (const cpx<T>*)tw);
  return hipGetLastError();
}

hipError_t mixed_row_r2c(Prec p, const MixedLine& ml, int nlines, const void* in, void* out, const void* tw,
                         hipStream_t s) {
  return p == P32 ? mx_row_r2c<float>(ml, nlines, in, out, tw, s) : mx_row_r2c<double>(ml, nlines, in, out, tw, s);
}

template <typename T>
static hipError_t mx_row_c2r(const MixedLine& ml, int nlines, const void* in, void* out, double scale, const void* tw,
                             hipStream_t s) {
  const int W = lines_per_block<T>(ml.n);
  const size_t lds = lds_bytes<T>(W, ml.n);
  allow(k_mx_row_c2r<T>, lds);
  hipLaunchKernelGGL((k_mx_row_c2r<T>), dim3((nlines + W - 1) / W), dim3(kMxThreads), lds, s, (const cpx<T>*)in,
                     (T*)out, nlines, W, (T)scale, ml, (const cpx<T>*)tw);
  return hipGetLastError();
}

hipError_t mixed_row_c2r(Prec p, const MixedLine& ml, int nlines, const void* in, void* out, double scale,
                         const void* tw, hipStream_t s) {
  return p == P32 ? mx_row_c2r<float>(ml, nlines, in, out, scale, tw, s)
                  : mx_row_c2r<double>(ml, nlines, in, out, scale, tw, s);
}

template <typename T>
static hipError_t mx_nls_row(const MixedLine& ml, int nlines, int ny, FieldRef psi, int mode, double pc,
                             double scale, const void* tw, hipStream_t s, StatusRef st) {
  const int W = lines_per_block<T>(ml.n);
  const size_t lds = lds_bytes<T>(W, ml.n);
  const dim3 grid((nlines + W - 1) / W), block(kMxThreads);
  auto go = [&](auto k) {
    allow(k, lds);
    hipLaunchKernelGGL(k, grid, block, lds, s, psi, nlines, ny, W, (T)pc, (T)scale, ml, (const cpx<T>*)tw, st);
  };
  if (mode == 0) go(k_mx_nls_row<T, 0>);
  else if (mode == 1) go(k_mx_nls_row<T, 1>);
  else go(k_mx_nls_row<T, 2>);
  return hipGetLastError();
}

hipError_t mixed_nls_row(Prec p, const MixedLine& ml, int nlines, int ny, FieldRef psi, int mode, double phase_coef,
                         double scale, const void* tw, hipStream_t s, StatusRef st) {
  return p == P32 ? mx_nls_row<float>(ml, nlines, ny, psi, mode, phase_coef, scale, tw, s, st)
                  : mx_nls_row<double>(ml, nlines, ny, psi, mode, phase_coef, scale, tw, s, st);
}

template <typename T>
static hipError_t mx_nls_col(const MixedLine& ml, int nx, int nfields, FieldRef psi, const void* tw, const void* ex,
                             const void* ey, hipStream_t s) {
  const int W = lines_per_block<T>(ml.n);
  const size_t lds = lds_bytes<T>(W, ml.n);
  const int tiles = (nx + W - 1) / W;
  allow(k_mx_nls_col<T>, lds);
  hipLaunchKernelGGL((k_mx_nls_col<T>), dim3(tiles * nfields), dim3(kMxThreads), lds, s, psi, nx, tiles, W,
                     (T)(1.0 / ((double)nx * ml.n)), ml, (const cpx<T>*)tw, (const cpx<T>*)ex, (const cpx<T>*)ey);
  return hipGetLastError();
}

hipError_t mixed_nls_col(Prec p, const MixedLine& ml, int nx, int nfields, FieldRef psi, const void* tw,
                         const void* ex, const void* ey, hipStream_t s) {
  return p == P32 ? mx_nls_col<float>(ml, nx, nfields, psi, tw, ex, ey, s)
                  : mx_nls_col<double>(ml, nx, nfields, psi, tw, ex, ey, s);
}

template <typename T>
static hipError_t mx_cq(const MixedLine& mlx, const MixedLine& mly, int nfields, const void* psi, void* spec,
                        double* row_part, double* col_part, const void* twx, const void* twy, double kx0, double ky0,
                        hipStream_t s) {
  const int nx = mlx.n, ny = mly.n;
  allow(k_mx_cq_row<T>, lds_bytes<T>(1, nx));
  hipLaunchKernelGGL((k_mx_cq_row<T>), dim3(nfields * ny), dim3(kMxThreads), lds_bytes<T>(1, nx), s,
                     (const cpx<T>*)psi, (cpx<T>*)spec, nfields * ny, row_part, mlx, (const cpx<T>*)twx);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  allow(k_mx_cq_col<T>, lds_bytes<T>(1, ny));
  hipLaunchKernelGGL((k_mx_cq_col<T>), dim3(nfields * nx), dim3(kMxThreads), lds_bytes<T>(1, ny), s,
                     (const cpx<T>*)spec, nx, col_part, mly, (const cpx<T>*)twy, kx0, ky0);
  return hipGetLastError();
}

hipError_t mixed_nls_cq(Prec p, const MixedLine& mlx, const MixedLine& mly, int nfields, const void* psi, void* spec,
                        double* row_part, double* col_part, const void* twx, const void* twy, double kx0, double ky0,
                        hipStream_t s) {
  return p == P32 ? mx_cq<float>(mlx, mly, nfields, psi, spec, row_part, col_part, twx, twy, kx0, ky0, s)
                  : mx_cq<double>(mlx, mly, nfields, psi, spec, row_part, col_part, twx, twy, kx0, ky0, s);
}

}  // namespace pst
