// NLS conserved quantities (eq. nlsmassenergy with nonlinearity g):
//   mass   = dx dy sum |psi|^2
//   energy = (1/2) lx ly/(nx ny)^2 sum |k|^2 |psi_hat|^2 + (g/4) dx dy sum |psi|^4
// All sums accumulate in double in a fixed order: per thread, per line
// (fixed tree), then per field (fixed tree).
#include "kernels.hpp"
#include "launch.hpp"

namespace pst {

template <typename T, int N>
__global__ __launch_bounds__((RowGeom<T, N>::THREADS)) void k_nls_cq_row(
    const cpx<T>* psi, cpx<T>* spec, int nlines, double* part, const cpx<T>* __restrict__ tw) {
  using G = RowGeom<T, N>;
  extern __shared__ char smem[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem);
  __shared__ double red[G::THREADS];
  const int lid = threadIdx.x / G::TL, t = threadIdx.x % G::TL;
  const int line = blockIdx.x * G::LPB + lid;
  const bool valid = line < nlines;
  cpx<T>* L = lds + lid * lds_line_stride<T>(N);
  cpx<T> v[G::R];
  double m2 = 0.0, m4 = 0.0;
#pragma unroll
  for (int s = 0; s < G::R; ++s) {
    v[s] = valid ? psi[(size_t)line * N + t + s * G::TL] : cpx<T>{0, 0};
    const double a = (double)v[s].re * v[s].re + (double)v[s].im * v[s].im;
    m2 += a;
    m4 += a * a;
  }
  m2 = line_sum(red, lid, t, G::TL, m2);
  m4 = line_sum(red, lid, t, G::TL, m4);
  if (valid && t == 0) {
    store1(part + 2 * (size_t)line, m2);
    store1(part + 2 * (size_t)line + 1, m4);
  }
  line_fft<N, false>(v, L, t, tw);
  if (valid) {
#pragma unroll
    for (int s = 0; s < G::R; ++s) gstore(spec + ((size_t)line * N + t + s * G::TL), v[s]);
  }
}

template <typename T, int N, int WT>
__global__ __launch_bounds__((WT * (N / line_radix(N)))) void k_nls_cq_col(cpx<T>* spec, int nx, int tiles_per_field,
                                                     double* part, const cpx<T>* __restrict__ tw,
                                                     double kx0, double ky0) {
  using G = ColGeom<T, N, WT>;
  extern __shared__ char smem[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem);
  __shared__ double red[1024];
  const int c = threadIdx.x % WT, t = threadIdx.x / WT;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int field = tile / tiles_per_field;
  const int col = (tile % tiles_per_field) * WT + c;
  const bool valid = col < nx;
  cpx<T>* base = spec + (size_t)field * N * nx + col;
  cpx<T>* L = lds + c;
  cpx<T> v[G::R];
#pragma unroll
  for (int s = 0; s < G::R; ++s) v[s] = valid ? base[(size_t)(t + s * G::TL) * nx] : cpx<T>{0, 0};
  line_fft<N, false, WT>(v, L, t, tw);
  const int mx = col < nx / 2 ? col : col - nx;
  const double kx = kx0 * mx;
  double acc = 0.0;
#pragma unroll
  for (int s = 0; s < G::R; ++s) {
    const int e = t + s * G::TL;
    const int my = e < N / 2 ? e : e - N;
    const double ky = ky0 * my;
    acc += (kx * kx + ky * ky) * ((double)v[s].re * v[s].re + (double)v[s].im * v[s].im);
  }
  acc = line_sum(red, c, t, G::TL, acc);
  if (valid && t == 0) part[(size_t)field * nx + col] = acc;
}

// One block per field; 256 threads each sum a fixed strided subset, then a
// fixed tree.
__global__ __launch_bounds__(256) void k_nls_cq_finish(int ny, int nx, const double* row_part,
                                                       const double* col_part, double dxdy,
                                                       double kin_coef, double g, double* out,
                                                       int* status) {
  __shared__ double red[256];
  const int f = blockIdx.x, t = threadIdx.x;
  double a = 0.0, b = 0.0, c = 0.0;
  for (int i = t; i < ny; i += 256) {
    a += row_part[2 * ((size_t)f * ny + i)];
    b += row_part[2 * ((size_t)f * ny + i) + 1];
  }
  for (int i = t; i < nx; i += 256) c += col_part[(size_t)f * nx + i];
  a = line_sum(red, 0, t, 256, a);
  b = line_sum(red, 0, t, 256, b);
  c = line_sum(red, 0, t, 256, c);
  if (t == 0) {
    const double mass = dxdy * a;
    const double kin = kin_coef * c;
    const double pot = 0.25 * g * dxdy * b;
    store1(out + 4 * f + 0, mass);
    store1(out + 4 * f + 1, kin + pot);
    store1(out + 4 * f + 2, kin);
    store1(out + 4 * f + 3, pot);
    if (!isfinite(mass) || !isfinite(kin + pot)) atomicOr(status, (int)ST_NONFINITE);
  }
}

template <typename T>
static hipError_t cq_row(int nx, int nlines, const void* psi, void* spec, double* part, const void* tw,
                         hipStream_t s) {
  bool ok = dispatch_n(nx, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    using G = RowGeom<T, N>;
    const int grid = (nlines + G::LPB - 1) / G::LPB;
    allow_lds((k_nls_cq_row<T, N>), G::LDS_BYTES);
    hipLaunchKernelGGL((k_nls_cq_row<T, N>), dim3(grid), dim3(G::THREADS), G::LDS_BYTES, s,
                       (const cpx<T>*)psi, (cpx<T>*)spec, nlines, part, (const cpx<T>*)tw);
  });
  return ok ? hipGetLastError() : hipErrorInvalidValue;
}

hipError_t nls_cq_row(Prec p, int nx, int nlines, const void* psi, void* spec, double* part,
                      const void* tw, hipStream_t s) {
  return p == P32 ? cq_row<float>(nx, nlines, psi, spec, part, tw, s)
                  : cq_row<double>(nx, nlines, psi, spec, part, tw, s);
}

template <typename T>
static hipError_t cq_col(int ny, int nx, int nfields, void* spec, double* part, const void* tw,
                         double kx0, double ky0, int W, hipStream_t s) {
  bool ok = false;
  dispatch_n(ny, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    ok = dispatch_w<T, N>(W, [&](auto wc) {
    constexpr int WT = decltype(wc)::value;
    using G = ColGeom<T, N, WT>;
    const int tiles = (nx + WT - 1) / WT;
    allow_lds((k_nls_cq_col<T, N, WT>), G::LDS_BYTES);
    hipLaunchKernelGGL((k_nls_cq_col<T, N, WT>), dim3(tiles * nfields), dim3(G::THREADS), G::LDS_BYTES,
                       s, (cpx<T>*)spec, nx, tiles, part, (const cpx<T>*)tw, kx0, ky0);
    });
  });
  return ok ? hipGetLastError() : hipErrorInvalidValue;
}

hipError_t nls_cq_col(Prec p, int ny, int nx, int nfields, void* spec, double* part, const void* tw,
                      double kx0, double ky0, int W, hipStream_t s) {
  return p == P32 ? cq_col<float>(ny, nx, nfields, spec, part, tw, kx0, ky0, W, s)
                  : cq_col<double>(ny, nx, nfields, spec, part, tw, kx0, ky0, W, s);
}

hipError_t nls_cq_finish(int nfields, int ny, int nx, const double* row_part, const double* col_part,
                         double dxdy, double kin_coef, double g, double* out, int* status,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_nls_cq_finish, dim3(nfields), dim3(256), 0, s, ny, nx, row_part, col_part, dxdy,
                     kin_coef, g, out, status);
  return hipGetLastError();
}

}  // namespace pst
