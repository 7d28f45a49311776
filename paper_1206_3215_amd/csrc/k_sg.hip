// Sine-Gordon passes: the three-level scheme of Section "A Numerical Method
// for the Sine-Gordon Equation" (Laplacian sign as in eq. sg).  In Fourier
// space, with a = |k|^2 dt^2 / 4,
//     u^{n+1} - 2u^n + u^{n-1} = (c1 - 2) u^n - c2 FFT(sin u^n),
//     c1 - 2 = -4a/(1 + a),  c2 = dt^2/(1 + a).
// The state is carried as u^n and the increment d^n = u^n - u^{n-1} in
// physical space; only the small second difference goes through the
// transforms.  (Forming u^{n+1} = c1 u^n - u^{n-1} through an FFT round trip
// instead lets single-precision rounding that varies slowly from step to
// step drive the slow modes, whose response grows like 1/theta^2 for a mode
// rotating by theta per step.)
//   column pass (half-width columns): W = iFFT_y((c1-2) FFT_y(U) - c2 FFT_y(S))
//   row pass (pairs of real rows):    d^{n+1} = d^n + C2R_x(W);
//                                     u^{n+1} = u^n + d^{n+1};
//                                     U = R2C_x(u^{n+1}); S = R2C_x(sin u^{n+1})
// The row pass's split leaves 2U, 2S; that factor and the unnormalised
// transforms' 1/(nx ny) are folded into the column coefficients (sc).
#include "kernels.hpp"
#include "launch.hpp"

namespace pst {

// ENTRY: U, S from u_old and, if d_out != NULL, d_out = u_old - d_old (the
//        increment from the two caller levels u_curr, u_prev).
// STEP:  d_out = d_old + C2R(W), u_out = u_old + d_out, then U, S.
// FINAL: d = alpha d_old + C2R(W), u_out = u_old + d, prev_out = u_old.
enum { SG_ENTRY = 0, SG_STEP = 1, SG_FINAL = 2 };

__device__ __forceinline__ float sin_of(float x) { return sin_f32(x); }
__device__ __forceinline__ double sin_of(double x) { return sin(x); }

template <typename T, int N, int MODE>
__global__ __launch_bounds__((RowGeom<T, N>::THREADS)) void k_sg_row(
    const cpx<T>* W, FieldRef u_old_f, FieldRef d_old_f, T alpha, FieldRef u_out_f, FieldRef d_out_f,
    FieldRef prev_out_f, cpx<T>* U, cpx<T>* S, int nlines, int lny, const cpx<T>* __restrict__ tw, StatusRef st) {
  using G = RowGeom<T, N>;
  constexpr int H = N / 2 + 1;
  extern __shared__ char smem[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem);
  const int lid = threadIdx.x / G::TL, t = threadIdx.x % G::TL;
  const int pair = blockIdx.x * G::LPB + lid;
  const int la = 2 * pair, lb = 2 * pair + 1;
  const bool va = la < nlines, vb = lb < nlines;
  cpx<T>* L = lds + lid * lds_line_stride<T>(N);
  const int r0 = 2 * blockIdx.x * G::LPB;
  // U, S, W hold the rows of each pair interleaved (see ColArr)
  // (line counts are even: rows a and b of a pair are present together, and
  // the interleaved layout puts their elements side by side from oa)
  const unsigned oa = pair_row_off_il<T, N>(la - r0, va && vb);
  // rows a, b are rows y, y+1 of field f; offsets are relative to each field
  const int f = la >> lny;
  const size_t ra = (size_t)(la & ((1 << lny) - 1)) * N, rb = ra + N;
  gptr<const T> u_old = field<const T>(u_old_f, f);
  gptr<const T> d_old = field<const T>(d_old_f, f);
  gptr<T> u_out = field<T>(u_out_f, f);
  gptr<T> d_out = field<T>(d_out_f, f);
  gptr<T> prev_out = field<T>(prev_out_f, f);
  cpx<T> u[G::R];
  if constexpr (MODE == SG_ENTRY) {
#pragma unroll
    for (int s = 0; s < G::R; ++s) {
      const int e = t + s * G::TL;
      const T ua = va ? u_old[ra + e] : T(0), ub = vb ? u_old[rb + e] : T(0);
      if (d_out_f.base != nullptr || d_out_f.table != nullptr) {
        if (va) d_out[ra + e] = ua - d_old[ra + e];
        if (vb) d_out[rb + e] = ub - d_old[rb + e];
      }
      u[s] = cpx<T>{ua, ub};
    }
  } else {
    const FieldBuf wb = pair_rows<T, N>(W, r0, 2 * G::LPB);
    load_pair_spectrum_il<T, N>(u, wb, oa, t, T(1));
    line_fft<N, true>(u, L, t, tw);
    mem_fence_compiler();
#pragma unroll
    for (int s = 0; s < G::R; ++s) {
      const int e = t + s * G::TL;
      const T oa = va ? u_old[ra + e] : T(0), ob = vb ? u_old[rb + e] : T(0);
      const T pa = va ? d_old[ra + e] : T(0), pb = vb ? d_old[rb + e] : T(0);
      const T da = alpha * pa + u[s].re, db = alpha * pb + u[s].im;
      u[s] = cpx<T>{oa + da, ob + db};
      if constexpr (MODE == SG_FINAL) {
        if (va) prev_out[ra + e] = oa;
        if (vb) prev_out[rb + e] = ob;
      } else {
        if (va) d_out[ra + e] = da;
        if (vb) d_out[rb + e] = db;
      }
      if (va) u_out[ra + e] = u[s].re;
      if (vb) u_out[rb + e] = u[s].im;
    }
    if constexpr (MODE == SG_FINAL) {
      // the last pass of a call reports a field holding a non-finite value
      bool bad = false;
#pragma unroll
      for (int s = 0; s < G::R; ++s) bad = bad || (va && !isfinite(u[s].re)) || (vb && !isfinite(u[s].im));
      // a wave spans 128/TL rows of whole pairs, all in one field when ny >= 128/TL
      latch_nonfinite(bad, st, f, G::TL >= 64 || (1 << lny) * G::TL >= 128);
    }
  }
  if constexpr (MODE == SG_STEP) {
    // S from a second line array, u kept in registers for U (the kernel's
    // occupancy is already set above 128 registers, so the second array
    // costs no waves and saves reading u^{n+1} back)
    cpx<T> sn[G::R];
#pragma unroll
    for (int s = 0; s < G::R; ++s) sn[s] = cpx<T>{sin_of(u[s].re), sin_of(u[s].im)};
    line_fft<N, false>(sn, L, t, tw);
    const FieldBuf sb = pair_rows<T, N>(S, r0, 2 * G::LPB);
    store_pair_halves_il<T, N>(sn, L, t, sb, oa);
    line_fft<N, false>(u, L, t, tw);
    const FieldBuf ub = pair_rows<T, N>(U, r0, 2 * G::LPB);
    store_pair_halves_il<T, N>(u, L, t, ub, oa);
  } else if constexpr (MODE == SG_ENTRY) {
    // S first, from sin(u) in place; u is then read again from the input, so
    // only one line array is live at a time.
#pragma unroll
    for (int s = 0; s < G::R; ++s) u[s] = cpx<T>{sin_of(u[s].re), sin_of(u[s].im)};
    line_fft<N, false>(u, L, t, tw);
    const FieldBuf sb = pair_rows<T, N>(S, r0, 2 * G::LPB);
    store_pair_halves_il<T, N>(u, L, t, sb, oa);
    mem_fence_compiler();
#pragma unroll
    for (int s = 0; s < G::R; ++s) {
      const int e = t + s * G::TL;
      u[s] = cpx<T>{va ? u_old[ra + e] : T(0), vb ? u_old[rb + e] : T(0)};
    }
    line_fft<N, false>(u, L, t, tw);
    const FieldBuf ub = pair_rows<T, N>(U, r0, 2 * G::LPB);
    store_pair_halves_il<T, N>(u, L, t, ub, oa);
  }
}

// Column pass over the nx/2+1 half-spectrum columns.
template <typename T, int N, int WT>
__global__ __launch_bounds__((WT * (N / line_radix(N)))) void k_sg_col(const cpx<T>* U, const cpx<T>* S, cpx<T>* W,
                                                                       int ncols, int tiles_per_field,
                                                                       const cpx<T>* __restrict__ tw, T kx0, T ky0,
                                                                       T dt2q, T cnum, T c2num, T sc) {
  using G = ColGeom<T, N, WT>;
  extern __shared__ char smem[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem);
  const int c = threadIdx.x % WT, t = threadIdx.x / WT;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int field = tile / tiles_per_field;
  const int col = (tile % tiles_per_field) * WT + c;
  const bool valid = col < ncols;
  const ColArr<T, true> Ua(U, field, N, ncols, col, valid, t, G::TL), Sa(S, field, N, ncols, col, valid, t, G::TL),
      Wa(W, field, N, ncols, col, valid, t, G::TL);
  cpx<T>* L = lds + c;
  const T kx = kx0 * (T)col;
  const T kx2 = kx * kx;
  // (c1 - 2) and c2 of mode e of this column: step c1 - 2 = -4a/(1+a)
  // (cnum 2), start c1 - 1 = -2a/(1+a) (cnum 1)
  auto coef = [&](int s, T& c1m, T& c2) {
    const int e = t + s * G::TL;
    const T ky = ky0 * (T)(e < N / 2 ? e : e - N);
    const T a = (kx2 + ky * ky) * dt2q;
    const T inv = T(1) / (T(1) + a);
    c1m = T(-2) * cnum * a * inv * sc;
    c2 = c2num * inv * sc;
  };
  cpx<T> u[G::R], s_[G::R];
#pragma unroll
  for (int s = 0; s < G::R; ++s) u[s] = Ua.ld(s);
  line_fft<N, false, WT>(u, L, t, tw);
  mem_fence_compiler();
#pragma unroll
  for (int s = 0; s < G::R; ++s) s_[s] = Sa.ld(s);
  line_fft<N, false, WT>(s_, L, t, tw);
#pragma unroll
  for (int s = 0; s < G::R; ++s) {
    T c1m, c2;
    coef(s, c1m, c2);
    u[s] = cpx<T>{c1m * u[s].re - c2 * s_[s].re, c1m * u[s].im - c2 * s_[s].im};
  }
  line_fft<N, true, WT>(u, L, t, tw);
#pragma unroll
  for (int s = 0; s < G::R; ++s) Wa.st(s, u[s]);
}

// ----------------------------------------------------------- Hamiltonian ---
// Row pass: per row pair, sums of ((u1-u0)/dt)^2 -> part[4p], and of
// sin^2(u1/2) + sin^2(u0/2) = ((1-cos u1) + (1-cos u0))/2 -> part[4p+1]
// (double precision), and the x-transform of ubar = (u0+u1)/2 (times 2).
template <typename T, int N>
__global__ __launch_bounds__((RowGeom<T, N>::THREADS)) void k_sg_h_row(
    const T* f0, const T* f1, cpx<T>* UB, double* part, int nlines, double inv_dt,
    const cpx<T>* __restrict__ tw) {
  using G = RowGeom<T, N>;
  constexpr int H = N / 2 + 1;
  extern __shared__ char smem[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem);
  __shared__ double red[G::THREADS];
  const int lid = threadIdx.x / G::TL, t = threadIdx.x % G::TL;
  const int pair = blockIdx.x * G::LPB + lid;
  const int la = 2 * pair, lb = 2 * pair + 1;
  const bool va = la < nlines, vb = lb < nlines;
  cpx<T>* L = lds + lid * lds_line_stride<T>(N);
  const T* ra = f0 + (size_t)la * N;
  const T* rb = f0 + (size_t)lb * N;
  const T* qa = f1 + (size_t)la * N;
  const T* qb = f1 + (size_t)lb * N;
  // FP64 sums in a rolled loop (one value's sines live at a time)
  double kin = 0.0, pot = 0.0;
#pragma unroll 1
  for (int s = 0; s < G::R; ++s) {
    const int e = t + s * G::TL;
    const double a0 = va ? (double)ra[e] : 0.0, a1 = va ? (double)qa[e] : 0.0;
    const double b0 = vb ? (double)rb[e] : 0.0, b1 = vb ? (double)qb[e] : 0.0;
    const double da = (a1 - a0) * inv_dt, db = (b1 - b0) * inv_dt;
    kin += da * da + db * db;
    const double sa0 = sin(0.5 * a0), sa1 = sin(0.5 * a1), sb0 = sin(0.5 * b0), sb1 = sin(0.5 * b1);
    pot += sa0 * sa0 + sa1 * sa1 + sb0 * sb0 + sb1 * sb1;
  }
  cpx<T> ub[G::R];
#pragma unroll
  for (int s = 0; s < G::R; ++s) {
    const int e = t + s * G::TL;
    const double a0 = va ? (double)ra[e] : 0.0, a1 = va ? (double)qa[e] : 0.0;
    const double b0 = vb ? (double)rb[e] : 0.0, b1 = vb ? (double)qb[e] : 0.0;
    ub[s] = cpx<T>{(T)(0.5 * (a0 + a1)), (T)(0.5 * (b0 + b1))};
  }
  kin = line_sum(red, lid, t, G::TL, kin);
  pot = line_sum(red, lid, t, G::TL, pot);
  if (t == 0 && va) {
    store1(part + 4 * (size_t)pair, kin);
    store1(part + 4 * (size_t)pair + 1, pot);
  }
  line_fft<N, false>(ub, L, t, tw);
  store_pair_halves<T, N>(ub, L, t, UB + (size_t)la * H, UB + (size_t)lb * H, va, vb);
}

// Column pass: sum over the half spectrum of w(mx) |k|^2 |2 ubar_hat|^2 with
// w = 1 on the self-conjugate columns mx = 0, nx/2 and 2 elsewhere.
template <typename T, int N, int WT>
__global__ __launch_bounds__((WT * (N / line_radix(N)))) void k_sg_h_col(cpx<T>* UB, double* part, int ncols, int nx,
                                                   int tiles_per_field, const cpx<T>* __restrict__ tw,
                                                   double kx0, double ky0) {
  using G = ColGeom<T, N, WT>;
  extern __shared__ char smem[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem);
  __shared__ double red[1024];
  const int c = threadIdx.x % WT, t = threadIdx.x / WT;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int field = tile / tiles_per_field;
  const int col = (tile % tiles_per_field) * WT + c;
  const bool valid = col < ncols;
  const ColArr<T> UBa(UB, field, N, ncols, col, valid, t, G::TL);
  cpx<T>* L = lds + c;
  cpx<T> v[G::R];
#pragma unroll
  for (int s = 0; s < G::R; ++s) v[s] = UBa.ld(s);
  line_fft<N, false, WT>(v, L, t, tw);
  const double kx = kx0 * col;
  const double w = (col == 0 || col == nx / 2) ? 1.0 : 2.0;
  double acc = 0.0;
#pragma unroll
  for (int s = 0; s < G::R; ++s) {
    const int e = t + s * G::TL;
    const double ky = ky0 * (e < N / 2 ? e : e - N);
    acc += (kx * kx + ky * ky) * ((double)v[s].re * v[s].re + (double)v[s].im * v[s].im);
  }
  acc = line_sum(red, c, t, G::TL, acc * w);
  if (valid && t == 0) part[(size_t)field * ncols + col] = acc;
}

__global__ __launch_bounds__(256) void k_sg_h_finish(int npairs, int ncols, const double* row_part,
                                                     const double* col_part, double dxdy, double grad_coef,
                                                     double* out, int* status) {
  __shared__ double red[256];
  const int f = blockIdx.x, t = threadIdx.x;
  double a = 0.0, b = 0.0, c = 0.0;
  for (int i = t; i < npairs; i += 256) {
    a += row_part[4 * ((size_t)f * npairs + i)];
    b += row_part[4 * ((size_t)f * npairs + i) + 1];
  }
  for (int i = t; i < ncols; i += 256) c += col_part[(size_t)f * ncols + i];
  a = line_sum(red, 0, t, 256, a);
  b = line_sum(red, 0, t, 256, b);
  c = line_sum(red, 0, t, 256, c);
  if (t == 0) {
    const double kin = 0.5 * dxdy * a, pot = dxdy * b, grad = grad_coef * c;
    store1(out + 4 * f + 0, kin + grad + pot);
    store1(out + 4 * f + 1, kin);
    store1(out + 4 * f + 2, grad);
    store1(out + 4 * f + 3, pot);
    if (!isfinite(kin + grad + pot)) atomicOr(status, (int)ST_NONFINITE);
  }
}

// ----------------------------------------------------------- launchers ---
template <typename T>
static hipError_t row(int mode, int nx, int nlines, int ny, const void* W, FieldRef u_old, FieldRef d_old,
                      double alpha, FieldRef u_out, FieldRef d_out, FieldRef prev_out, void* U, void* S,
                      const void* tw, hipStream_t s, StatusRef st) {
  if (nlines % 2 != 0) return hipErrorInvalidValue;  // the kernels take rows in pairs
  bool ok = dispatch_n(nx, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    using G = RowGeom<T, N>;
    const int grid = ((nlines + 1) / 2 + G::LPB - 1) / G::LPB;
    auto go = [&](auto kern) {
      allow_lds(kern, G::LDS_BYTES);
      hipLaunchKernelGGL(kern, dim3(grid), dim3(G::THREADS), G::LDS_BYTES, s, (const cpx<T>*)W, u_old, d_old,
                         (T)alpha, u_out, d_out, prev_out, (cpx<T>*)U, (cpx<T>*)S, nlines, ilog2c(ny),
                         (const cpx<T>*)tw, st);
    };
    if (mode == SG_ENTRY) go(k_sg_row<T, N, SG_ENTRY>);
    else if (mode == SG_STEP) go(k_sg_row<T, N, SG_STEP>);
    else go(k_sg_row<T, N, SG_FINAL>);
  });
  return ok ? hipGetLastError() : hipErrorInvalidValue;
}

hipError_t sg_row(Prec p, int mode, int nx, int nlines, int ny, const void* W, FieldRef u_old, FieldRef d_old,
                  double alpha, FieldRef u_out, FieldRef d_out, FieldRef prev_out, void* U, void* S,
                  const void* tw, hipStream_t s, StatusRef st) {
  return p == P32 ? row<float>(mode, nx, nlines, ny, W, u_old, d_old, alpha, u_out, d_out, prev_out, U, S, tw, s, st)
                  : row<double>(mode, nx, nlines, ny, W, u_old, d_old, alpha, u_out, d_out, prev_out, U, S, tw, s,
                                st);
}

template <typename T>
static hipError_t col(int ny, int nx, int nfields, const void* U, const void* S, void* W, const void* tw,
                      double kx0, double ky0, double dt2q, double cnum, double c2num, double sc, int Wt,
                      hipStream_t s) {
  bool ok = false;
  dispatch_n(ny, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    ok = dispatch_w<T, N>(Wt, [&](auto wc) {
    constexpr int WT = decltype(wc)::value;
    using G = ColGeom<T, N, WT>;
    const int ncols = nx / 2 + 1;
    const int tiles = (ncols + WT - 1) / WT;
    allow_lds(k_sg_col<T, N, WT>, G::LDS_BYTES);
    hipLaunchKernelGGL((k_sg_col<T, N, WT>), dim3(tiles * nfields), dim3(G::THREADS), G::LDS_BYTES, s,
                       (const cpx<T>*)U, (const cpx<T>*)S, (cpx<T>*)W, ncols, tiles, (const cpx<T>*)tw,
                       (T)kx0, (T)ky0, (T)dt2q, (T)cnum, (T)c2num, (T)sc);
    });
  });
  return ok ? hipGetLastError() : hipErrorInvalidValue;
}

hipError_t sg_col(Prec p, int ny, int nx, int nfields, const void* U, const void* S, void* W, const void* tw,
                  double kx0, double ky0, double dt2q, double cnum, double c2num, double sc, int Wt,
                  hipStream_t s) {
  return p == P32 ? col<float>(ny, nx, nfields, U, S, W, tw, kx0, ky0, dt2q, cnum, c2num, sc, Wt, s)
                  : col<double>(ny, nx, nfields, U, S, W, tw, kx0, ky0, dt2q, cnum, c2num, sc, Wt, s);
}

template <typename T>
static hipError_t hrow(int nx, int nlines, const void* f0, const void* f1, void* UB, double* part,
                       double inv_dt, const void* tw, hipStream_t s) {
  bool ok = dispatch_n(nx, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    using G = RowGeom<T, N>;
    const int grid = ((nlines + 1) / 2 + G::LPB - 1) / G::LPB;
    allow_lds(k_sg_h_row<T, N>, G::LDS_BYTES);
    hipLaunchKernelGGL((k_sg_h_row<T, N>), dim3(grid), dim3(G::THREADS), G::LDS_BYTES, s, (const T*)f0,
                       (const T*)f1, (cpx<T>*)UB, part, nlines, inv_dt, (const cpx<T>*)tw);
  });
  return ok ? hipGetLastError() : hipErrorInvalidValue;
}

hipError_t sg_h_row(Prec p, int nx, int nlines, const void* f0, const void* f1, void* UB, double* part,
                    double inv_dt, const void* tw, hipStream_t s) {
  return p == P32 ? hrow<float>(nx, nlines, f0, f1, UB, part, inv_dt, tw, s)
                  : hrow<double>(nx, nlines, f0, f1, UB, part, inv_dt, tw, s);
}

template <typename T>
static hipError_t hcol(int ny, int nx, int nfields, void* UB, double* part, const void* tw, double kx0,
                       double ky0, int Wt, hipStream_t s) {
  bool ok = false;
  dispatch_n(ny, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    ok = dispatch_w<T, N>(Wt, [&](auto wc) {
    constexpr int WT = decltype(wc)::value;
    using G = ColGeom<T, N, WT>;
    const int ncols = nx / 2 + 1;
    const int tiles = (ncols + WT - 1) / WT;
    allow_lds(k_sg_h_col<T, N, WT>, G::LDS_BYTES);
    hipLaunchKernelGGL((k_sg_h_col<T, N, WT>), dim3(tiles * nfields), dim3(G::THREADS), G::LDS_BYTES, s,
                       (cpx<T>*)UB, part, ncols, nx, tiles, (const cpx<T>*)tw, kx0, ky0);
    });
  });
  return ok ? hipGetLastError() : hipErrorInvalidValue;
}

hipError_t sg_h_col(Prec p, int ny, int nx, int nfields, void* UB, double* part, const void* tw, double kx0,
                    double ky0, int Wt, hipStream_t s) {
  return p == P32 ? hcol<float>(ny, nx, nfields, UB, part, tw, kx0, ky0, Wt, s)
                  : hcol<double>(ny, nx, nfields, UB, part, tw, kx0, ky0, Wt, s);
}

hipError_t sg_h_finish(int nfields, int npairs, int ncols, const double* row_part, const double* col_part,
                       double dxdy, double grad_coef, double* out, int* status, hipStream_t s) {
  hipLaunchKernelGGL(k_sg_h_finish, dim3(nfields), dim3(256), 0, s, npairs, ncols, row_part, col_part, dxdy,
                     grad_coef, out, status);
  return hipGetLastError();
}

}  // namespace pst
