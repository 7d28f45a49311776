// Navier-Stokes passes: Crank-Nicolson in time with fixed-point iteration on
// the Jacobian (Section "A Numerical Method for the 2D Navier-Stokes
// Equation"), vorticity/stream function form, 2/3-rule dealiasing.
//
// With h = dt nu |k|^2 / 2 and N = FFT(J), J = psi_y omega_x - psi_x omega_y,
// the iterate of step n solves per mode
//     w^{k+1} = [(1 - h) w^n - dt/2 (N(w^n) + N(w^k))] / (1 + h).
// It is carried as the increment d = w - w^n:
//     q = -2 h w^n - dt/2 N(w^n)              (once per step)
//     d^{k+1} = (q - dt/2 N(w^k)) / (1 + h)
// so that single-precision coefficients near 1 never multiply the whole
// field; the fixed-point residual is then |d^{k+1} - d^k|^2 (Parseval).
//
// Spectral arrays are [field][ny][nx/2+1] complex; "hybrid" arrays hold the
// same layout transformed along x only.  Per iteration:
//   row pass (row pairs): each of the 4 derivative hybrids -> C2R_x of the
//       pair's two rows in one complex transform -> J = psi_y omega_x -
//       psi_x omega_y for both rows -> R2C_x of the two rows' J -> N hybrid
//       (times 2)
//   column pass: FFT_y(N hybrid) -> mask -> update d, residual ->
//       derivatives i ky psi, i kx w, i kx psi, i ky w of w = w^n + d ->
//       4 x iFFT_y -> derivative hybrids (scaled for the next C2R_x)
#include "kernels.hpp"
#include "launch.hpp"

namespace pst {

enum { NS_ENTRY = 0, NS_FIRST = 1, NS_ITER = 2, NS_EXIT = 3 };

// 1/x: the hardware reciprocal (about 1 ulp) in single precision, a
// correctly rounded division in double precision
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// A block's lines may span several fields; it may skip its work only when
// every field it touches has converged (the decision must be block-uniform).
__device__ __forceinline__ bool fields_done(const int* done, int f0, int f1) {
  for (int f = f0; f <= f1; ++f)
    if (!done[f]) return false;
  return true;
}

// Row pass.  FP32 lines of 2048 are held to 3 waves per SIMD (168
// registers): the 16-byte pair loads would otherwise take the kernel just
// past that and cost a wave; at this length the cap needs no spills (other
// lengths would spill, and run uncapped).
template <typename T, int N>
constexpr int ns_row_waves() {
  return sizeof(T) == 4 && N == 2048 ? 3 : 1;
}

template <typename T, int N>
__global__ __launch_bounds__((RowGeom<T, N>::THREADS)) __attribute__((amdgpu_waves_per_eu(ns_row_waves<T, N>()))) void k_ns_row(
    const cpx<T>* D, size_t dstride, cpx<T>* NH, int nlines, int ny, const int* done,
    const cpx<T>* __restrict__ tw) {
  using G = RowGeom<T, N>;
  constexpr int H = N / 2 + 1;
  extern __shared__ char smem[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem);
  const int lid = threadIdx.x / G::TL, t = threadIdx.x % G::TL;
  const int pair = blockIdx.x * G::LPB + lid;
  const int la = 2 * pair, lb = 2 * pair + 1;
  const bool va = la < nlines, vb = lb < nlines;
  if (done != nullptr) {
    const int p0 = blockIdx.x * G::LPB;
    const int l1 = min(2 * (p0 + G::LPB) - 1, nlines - 1);
    if (fields_done(done, (2 * p0) / ny, l1 / ny)) return;
  }
  cpx<T>* L = lds + lid * lds_line_stride<T>(N);
  // the block's rows through buffers (first row 2 p0, 2 LPB rows)
  const int r0 = 2 * blockIdx.x * G::LPB;
  const FieldBuf d0 = pair_rows<T, N>(D, r0, 2 * G::LPB), d1 = pair_rows<T, N>(D + dstride, r0, 2 * G::LPB),
                 d2 = pair_rows<T, N>(D + 2 * dstride, r0, 2 * G::LPB),
                 d3 = pair_rows<T, N>(D + 3 * dstride, r0, 2 * G::LPB), nh = pair_rows<T, N>(NH, r0, 2 * G::LPB);
  // the spectral work arrays hold the rows of each pair interleaved (ColArr)
  // (line counts are even: rows a and b of a pair are present together, and
  // the interleaved layout puts their elements side by side from oa)
  const unsigned oa = pair_row_off_il<T, N>(la - r0, va && vb);
  // Each derivative of the pair's two rows shares one complex transform,
  // z_q = D_q(row a) + i D_q(row b): the same field in both halves, so of
  // like magnitude (packing psi with omega, whose sizes differ by ~|k|^2,
  // would bury the stream-function derivatives in the vorticity
  // derivatives' rounding), and the two rows are adjacent in the
  // interleaved layout.  Then J_a = Re z0 Re z1 - Re z2 Re z3 and J_b the
  // same with the imaginary parts, and z = J_a + i J_b is transformed back.
  cpx<T> p[G::R], u[G::R], w[G::R];
  // each spectrum load takes an opaque copy of t, so that its per-element
  // offsets are computed where they are used rather than held in registers
  // across the transforms
  auto tk = [&]() {
    int x = t;
    asm volatile("" : "+v"(x));
    return x;
  };
  load_pair_spectrum_il<T, N>(u, d0, oa, tk(), T(1));  // psi_y
  line_fft<N, true>(u, L, t, tw);
  mem_fence_compiler();
  load_pair_spectrum_il<T, N>(w, d1, oa, tk(), T(1));  // omega_x
  line_fft<N, true>(w, L, t, tw);
#pragma unroll
  for (int s = 0; s < G::R; ++s) p[s] = cpx<T>{u[s].re * w[s].re, u[s].im * w[s].im};
  mem_fence_compiler();
  load_pair_spectrum_il<T, N>(u, d2, oa, tk(), T(1));  // psi_x
  line_fft<N, true>(u, L, t, tw);
  mem_fence_compiler();
  load_pair_spectrum_il<T, N>(w, d3, oa, tk(), T(1));  // omega_y
  line_fft<N, true>(w, L, t, tw);
#pragma unroll
  for (int s = 0; s < G::R; ++s) p[s] = cpx<T>{p[s].re - u[s].re * w[s].re, p[s].im - u[s].im * w[s].im};
  line_fft<N, false>(p, L, t, tw);
  store_pair_halves_il<T, N>(p, L, t, nh, oa);
}

struct NsColArgs {
  double kx0, ky0;  // 2 pi / lx, 2 pi / ly
  double hnu;       // dt nu / 2
  double qdt;       // dt / 2
  double nscale;    // 1/2: the row pass stores 2 x the Jacobian's transform
  double dscale;    // 1 / (nx ny): scale of the derivative hybrids
  int nx, kx_cut, ky_cut;
};

template <typename T, int N, int MODE, int WT>
__global__ __launch_bounds__((WT * (N / line_radix(N)))) void k_ns_col(const cpx<T>* NH, cpx<T>* WN, cpx<T>* Q, cpx<T>* DK,
                                                 cpx<T>* D, size_t dstride, cpx<T>* OUT, double* part,
                                                 int tiles_per_field, const int* gate, NsColArgs a,
                                                 const cpx<T>* __restrict__ tw) {
  using G = ColGeom<T, N, WT>;
  constexpr int MY = N;  // column length (ny)
  extern __shared__ char smem[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem);
  __shared__ double red[1024];
  const int ncols = a.nx / 2 + 1;
  const int c = threadIdx.x % WT, t = threadIdx.x / WT;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int field = tile / tiles_per_field;
  // a field the gate marks (converged, or waiting for the host) is left
  // alone; the decision is uniform, a block being one field
  if (gate != nullptr && gate[field]) return;
  const int col = (tile % tiles_per_field) * WT + c;
  // Later iterations leave out the Nyquist column x: it lies beyond the 2/3
  // cut, so N is masked there and the update, the derivatives and the
  // stored values equal the first iteration's (its residual term is zero);
  // the first iteration runs it at the end of the field's first tile
  const bool valid = col < (MODE == NS_ITER || MODE == NS_FIRST ? ncols - 1 : ncols);
  cpx<T>* L = lds + c;
  // columns past the end read zeros and store nothing (buffer range check)
  // work arrays in the pair-interleaved layout; the entry input (omega's
  // x-transform) and the exit output (read by the inverse real row pass) plain
  auto arr = [&](const cpx<T>* a) { return ColArr<T, true>(a, field, MY, ncols, col, valid, t, G::TL); };
  auto plain = [&](const cpx<T>* a) { return ColArr<T, false>(a, field, MY, ncols, col, valid, t, G::TL); };
  cpx<T> w[G::R], v[G::R];

  if constexpr (MODE == NS_EXIT) {
#pragma unroll
    for (int s = 0; s < G::R; ++s) v[s] = arr(WN).ld(s) + arr(DK).ld(s);
    line_fft<MY, true, WT>(v, L, t, tw);
    const ColArr<T> out = plain(OUT);
#pragma unroll
    for (int s = 0; s < G::R; ++s) out.st(s, v[s]);
    return;
  } else {
    const T kx = (T)(a.kx0 * col);
    const T kxd = (col == a.nx / 2) ? T(0) : kx;  // Nyquist dropped for first derivatives
    const bool xkeep = col <= a.kx_cut;
    double res = 0.0, ens = 0.0;
    // N hybrid -> spectrum (entry: omega's x-transform -> w^n)
#pragma unroll
    for (int s = 0; s < G::R; ++s) v[s] = MODE == NS_ENTRY ? plain(NH).ld(s) : arr(NH).ld(s);
    line_fft<MY, false, WT>(v, L, t, tw);
    mem_fence_compiler();
    const ColArr<T, true> wna = arr(WN), dka = arr(DK), qa = arr(Q);
    if constexpr (MODE == NS_ENTRY) {
#pragma unroll
      for (int s = 0; s < G::R; ++s) {
        w[s] = v[s];
        wna.st(s, v[s]);
        dka.st(s, cpx<T>{0, 0});
      }
    } else {
      const T hnu = (T)a.hnu, qdt = (T)a.qdt;
#pragma unroll
      for (int s = 0; s < G::R; ++s) {
        const int e = t + s * G::TL;
        const int my = e < MY / 2 ? e : e - MY;
        const T ky = (T)(a.ky0 * my);
        const T h = hnu * (kx * kx + ky * ky);
        const bool keep = xkeep && (my <= a.ky_cut && -my <= a.ky_cut);
        const cpx<T> nk = keep ? v[s] * (T)a.nscale : cpx<T>{0, 0};
        cpx<T> wn, q, dold;
        if (MODE == NS_FIRST) {
          // w^n = WN + (last step's increment); q = -2 h w^n - dt/2 N(w^n)
          wn = wna.ld(s) + dka.ld(s);
          q = cpx<T>{T(-2) * h * wn.re - qdt * nk.re, T(-2) * h * wn.im - qdt * nk.im};
          dold = cpx<T>{0, 0};
          wna.st(s, wn);
          qa.st(s, q);
        } else {
          wn = wna.ld(s);
          q = qa.ld(s);
          dold = dka.ld(s);
        }
        const T inv = T(1) / (T(1) + h);
        const cpx<T> dnew = cpx<T>{(q.re - qdt * nk.re) * inv, (q.im - qdt * nk.im) * inv};
        dka.st(s, dnew);
        const double dr = (double)dnew.re - (double)dold.re, di = (double)dnew.im - (double)dold.im;
        res += dr * dr + di * di;
        w[s] = wn + dnew;
        ens += (double)w[s].re * w[s].re + (double)w[s].im * w[s].im;
      }
    }
    // residual and |w|^2 partials, weighted for the half spectrum
    if (MODE != NS_ENTRY) {
      const double wt = (col == 0 || col == a.nx / 2) ? 1.0 : 2.0;
      res = line_sum(red, c, t, G::TL, res * wt);
      ens = line_sum(red, c, t, G::TL, ens * wt);
      if (valid && t == 0) {
        store1(part + 2 * ((size_t)field * ncols + col), res);
        store1(part + 2 * ((size_t)field * ncols + col) + 1, ens);
      }
    }
    // derivative hybrids of w: psi_y, omega_x, psi_x, omega_y
    const T dsc = (T)a.dscale;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      // the per-mode factors are recomputed for every derivative: held in
      // registers through the four transforms they would push the kernel
      // past 128 registers (opaque copy of t so they are not hoisted)
      int tq = t;
      asm volatile("" : "+v"(tq));
#pragma unroll
      for (int s = 0; s < G::R; ++s) {
        const int e = tq + s * G::TL;
        const int my = e < MY / 2 ? e : e - MY;
        const T ky = (T)(a.ky0 * my);
        const T kyd = (e == MY / 2) ? T(0) : ky;
        const T k2 = kx * kx + ky * ky;
        const T ik2 = k2 > T(0) ? dsc * recip(k2) : T(0);  // psi_hat = w / |k|^2, psi_hat(0) = 0
        const T f = q == 0 ? kyd * ik2 : q == 1 ? kxd * dsc : q == 2 ? kxd * ik2 : kyd * dsc;
        v[s] = mul_i(w[s]) * f;
      }
      line_fft<MY, true, WT>(v, L, t, tw);
      const ColArr<T, true> dq = arr(D + q * dstride);
#pragma unroll
      for (int s = 0; s < G::R; ++s) dq.st(s, v[s]);
      mem_fence_compiler();
    }
    if constexpr (MODE == NS_FIRST) {
      // A field's first tile also carries the x-Nyquist column (lane c = 0),
      // so that a field takes nx/2 / W tiles: N is masked there and both
      // x-derivatives vanish, so the column needs the update and two
      // inverse transforms, the same arithmetic as a tile of its own.
      if (tile % tiles_per_field == 0) {  // block-uniform
        // (its addressing is derived from an opaque copy of t after a
        // compiler fence, so none of it is computed early and held through
        // the transforms above)
        mem_fence_compiler();
        int tn = t;
        asm volatile("" : "+v"(tn));
        const int nh = ncols - 1;
        const bool pk = c == 0;
        const ColArr<T, true> wnn(WN, field, MY, ncols, nh, pk, tn, G::TL),
            dkn(DK, field, MY, ncols, nh, pk, tn, G::TL), qn(Q, field, MY, ncols, nh, pk, tn, G::TL);
        const T kxn = (T)(a.kx0 * nh);
        const T hnu = (T)a.hnu;
        double resn = 0.0, ensn = 0.0;
#pragma unroll
        for (int s = 0; s < G::R; ++s) {
          const int e = tn + s * G::TL;
          const int my = e < MY / 2 ? e : e - MY;
          const T ky = (T)(a.ky0 * my);
          const T h = hnu * (kxn * kxn + ky * ky);
          if (s % 4 == 0) mem_fence_compiler();  // at most four values' loads in flight
          const cpx<T> wn = wnn.ld(s) + dkn.ld(s);
          const cpx<T> q = cpx<T>{T(-2) * h * wn.re, T(-2) * h * wn.im};
          wnn.st(s, wn);
          qn.st(s, q);
          const T inv = T(1) / (T(1) + h);
          const cpx<T> dnew = cpx<T>{q.re * inv, q.im * inv};
          dkn.st(s, dnew);
          resn += (double)dnew.re * dnew.re + (double)dnew.im * dnew.im;
          w[s] = wn + dnew;
          ensn += (double)w[s].re * w[s].re + (double)w[s].im * w[s].im;
        }
        resn = line_sum(red, c, t, G::TL, resn);
        ensn = line_sum(red, c, t, G::TL, ensn);
        if (pk && t == 0) {
          store1(part + 2 * ((size_t)field * ncols + nh), resn);
          store1(part + 2 * ((size_t)field * ncols + nh) + 1, ensn);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const ColArr<T, true> dq(D + q * dstride, field, MY, ncols, nh, pk, tn, G::TL);
          if (q == 1 || q == 2) {
#pragma unroll
            for (int s = 0; s < G::R; ++s) dq.st(s, cpx<T>{0, 0});
            continue;
          }
          // (factors recomputed per derivative from an opaque copy of t, as
          // in the main loop, so they are not held through the transform)
          int tq = tn;
          asm volatile("" : "+v"(tq));
#pragma unroll
          for (int s = 0; s < G::R; ++s) {
            const int e = tq + s * G::TL;
            const int my = e < MY / 2 ? e : e - MY;
            const T ky = (T)(a.ky0 * my);
            const T kyd = (e == MY / 2) ? T(0) : ky;
            const T k2 = kxn * kxn + ky * ky;
            const T ik2 = k2 > T(0) ? dsc * recip(k2) : T(0);
            v[s] = mul_i(w[s]) * (q == 0 ? kyd * ik2 : kyd * dsc);
          }
          line_fft<MY, true, WT>(v, L, t, tw);
#pragma unroll
          for (int s = 0; s < G::R; ++s) dq.st(s, v[s]);
          mem_fence_compiler();
        }
      }
    }
  }
}

// Per field: residual r = dxdy/(nx ny) sum w |d^{k+1} - d^k|^2 against
// tol_eff = max(tol, fp_floor * integral omega^2); updates done/iters.
// first: the step's first iteration; fixed > 0: run exactly that many
// iterations.  With park != NULL the iterations of a step were queued ahead
// of time: a parked field (park[f] != 0) is skipped until the host resumes
// it, a field that converges records its count in maxit, and one that has
// not converged after the last queued iteration (last != 0) and has not
// reached max_iter is parked (done is set so that later iterations skip
// it, and park_step records the step of the chunk).
__global__ __launch_bounds__(256) void k_ns_finish(int ncols, const double* part, double vol, double tol,
                                                   double fp_floor, int max_iter, int fixed, int first,
                                                   int* done, int* iters, int* iters_out, double* resid,
                                                   int* status, int* const* fstat, NsPark pk) {
  __shared__ double red[256];
  const int f = blockIdx.x, t = threadIdx.x;
  if (pk.park != nullptr && pk.park[f]) return;
  if (!first && done[f]) return;
  double r = 0.0, z = 0.0;
  // after the first iteration the Nyquist column's residual term is zero and
  // its entry holds the first iteration's; its |w|^2 term is unchanged
  const int nres = first ? ncols : ncols - 1;
  for (int i = t; i < ncols; i += 256) {
    if (i < nres) r += part[2 * ((size_t)f * ncols + i)];
    z += part[2 * ((size_t)f * ncols + i) + 1];
  }
  r = line_sum(red, 0, t, 256, r);
  z = line_sum(red, 0, t, 256, z);
  if (t == 0) {
    const int it = first ? 1 : iters[f] + 1;
    iters[f] = it;
    const double res = vol * r, tol_eff = fmax(tol, fp_floor * vol * z);
    if (resid) resid[f] = res;
    bool fin;
    if (fixed > 0) {
      fin = it >= fixed;
    } else {
      fin = res < tol_eff;
      if (!fin && it >= max_iter) {
        fin = true;
        atomicOr(status, (int)ST_NOT_CONVERGED);
        if (fstat != nullptr && fstat[f] != nullptr) atomicOr(fstat[f], (int)ST_NOT_CONVERGED);
      }
    }
    if (!isfinite(res)) {
      fin = true;
      atomicOr(status, (int)ST_NONFINITE);
      if (fstat != nullptr && fstat[f] != nullptr) atomicOr(fstat[f], (int)ST_NONFINITE);
    }
    done[f] = fin ? 1 : 0;
    if (iters_out) iters_out[f] = it;
    if (pk.park != nullptr) {
      if (fin) {
        pk.maxit[f] = max(pk.maxit[f], it);
      } else if (pk.last) {
        pk.park[f] = 1;
        pk.park_step[f] = pk.step;
        done[f] = 1;
      }
    }
  }
}

// Diagnostics: energy (1/2) sum_{k != 0} |w|^2/|k|^2 and enstrophy
// (1/2) sum |w|^2 over the full spectrum (half-spectrum weights).
template <typename T, int N, int WT>
__global__ __launch_bounds__((WT * (N / line_radix(N)))) void k_ns_cq_col(const cpx<T>* XH, double* part, int nx, int tiles_per_field,
                                                    double kx0, double ky0, const cpx<T>* __restrict__ tw) {
  using G = ColGeom<T, N, WT>;
  extern __shared__ char smem[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem);
  __shared__ double red[1024];
  const int ncols = nx / 2 + 1;
  const int c = threadIdx.x % WT, t = threadIdx.x / WT;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int field = tile / tiles_per_field;
  const int col = (tile % tiles_per_field) * WT + c;
  const bool valid = col < ncols;
  const ColArr<T> xa(XH, field, N, ncols, col, valid, t, G::TL);
  cpx<T>* L = lds + c;
  cpx<T> v[G::R];
#pragma unroll
  for (int s = 0; s < G::R; ++s) v[s] = xa.ld(s);
  line_fft<N, false, WT>(v, L, t, tw);
  const double kx = kx0 * col;
  double en = 0.0, zz = 0.0;
#pragma unroll
  for (int s = 0; s < G::R; ++s) {
    const int e = t + s * G::TL;
    const double ky = ky0 * (e < N / 2 ? e : e - N);
    const double k2 = kx * kx + ky * ky;
    const double a2 = (double)v[s].re * v[s].re + (double)v[s].im * v[s].im;
    zz += a2;
    if (k2 > 0.0) en += a2 / k2;
  }
  const double wt = (col == 0 || col == nx / 2) ? 1.0 : 2.0;
  en = line_sum(red, c, t, G::TL, en * wt);
  zz = line_sum(red, c, t, G::TL, zz * wt);
  if (valid && t == 0) {
    store1(part + 2 * ((size_t)field * ncols + col), en);
    store1(part + 2 * ((size_t)field * ncols + col) + 1, zz);
  }
}

__global__ __launch_bounds__(256) void k_ns_cq_finish(int ncols, const double* part, double en_coef, double zz_coef,
                                                      double* out, int* status) {
  __shared__ double red[256];
  const int f = blockIdx.x, t = threadIdx.x;
  double a = 0.0, b = 0.0;
  for (int i = t; i < ncols; i += 256) {
    a += part[2 * ((size_t)f * ncols + i)];
    b += part[2 * ((size_t)f * ncols + i) + 1];
  }
  a = line_sum(red, 0, t, 256, a);
  b = line_sum(red, 0, t, 256, b);
  if (t == 0) {
    store1(out + 4 * f + 0, en_coef * a);
    store1(out + 4 * f + 1, zz_coef * b);
    store1(out + 4 * f + 2, 0.0);
    store1(out + 4 * f + 3, 0.0);
    if (!isfinite(a) || !isfinite(b)) atomicOr(status, (int)ST_NONFINITE);
  }
}

// ----------------------------------------------------------- launchers ---
template <typename T>
static hipError_t row(int nx, int nlines, int ny, const void* D, size_t dstride, void* NH, const int* done,
                      const void* tw, hipStream_t s) {
  if (nlines % 2 != 0) return hipErrorInvalidValue;  // the kernel takes rows in pairs
  bool ok = dispatch_n(nx, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    using G = RowGeom<T, N>;
    const int grid = ((nlines + 1) / 2 + G::LPB - 1) / G::LPB;
    allow_lds(k_ns_row<T, N>, G::LDS_BYTES);
    hipLaunchKernelGGL((k_ns_row<T, N>), dim3(grid), dim3(G::THREADS), G::LDS_BYTES, s, (const cpx<T>*)D, dstride,
                       (cpx<T>*)NH, nlines, ny, done, (const cpx<T>*)tw);
  });
  return ok ? hipGetLastError() : hipErrorInvalidValue;
}

hipError_t ns_row(Prec p, int nx, int nlines, int ny, const void* D, size_t dstride, void* NH, const int* done,
                  const void* tw, hipStream_t s) {
  return p == P32 ? row<float>(nx, nlines, ny, D, dstride, NH, done, tw, s)
                  : row<double>(nx, nlines, ny, D, dstride, NH, done, tw, s);
}

template <typename T>
static hipError_t col(int mode, int ny, int nfields, const NsPtrs& P, const NsScalars& S, const int* done,
                      const void* tw, int Wt, hipStream_t s) {
  bool ok = false;
  dispatch_n(ny, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    ok = dispatch_w<T, N>(Wt, [&](auto wc) {
    constexpr int WT = decltype(wc)::value;
    using G = ColGeom<T, N, WT>;
    const int ncols = S.nx / 2 + 1;
    const int nrun = mode == NS_ITER || mode == NS_FIRST ? ncols - 1 : ncols;  // see k_ns_col
    const int tiles = (nrun + WT - 1) / WT;
    NsColArgs a{S.kx0, S.ky0, S.hnu, S.qdt, S.nscale, S.dscale, S.nx, S.kx_cut, S.ky_cut};
    auto go = [&](auto kern) {
      allow_lds(kern, G::LDS_BYTES);
      hipLaunchKernelGGL(kern, dim3(tiles * nfields), dim3(G::THREADS), G::LDS_BYTES, s, (const cpx<T>*)P.NH,
                         (cpx<T>*)P.WN, (cpx<T>*)P.Q, (cpx<T>*)P.DK, (cpx<T>*)P.D, P.dstride, (cpx<T>*)P.OUT,
                         P.part, tiles, done, a, (const cpx<T>*)tw);
    };
    if (mode == NS_ENTRY) go(k_ns_col<T, N, NS_ENTRY, WT>);
    else if (mode == NS_FIRST) go(k_ns_col<T, N, NS_FIRST, WT>);
    else if (mode == NS_ITER) go(k_ns_col<T, N, NS_ITER, WT>);
    else go(k_ns_col<T, N, NS_EXIT, WT>);
    });
  });
  return ok ? hipGetLastError() : hipErrorInvalidValue;
}

hipError_t ns_col(Prec p, int mode, int ny, int nfields, const NsPtrs& P, const NsScalars& S, const int* done,
                  const void* tw, int Wt, hipStream_t s) {
  return p == P32 ? col<float>(mode, ny, nfields, P, S, done, tw, Wt, s)
                  : col<double>(mode, ny, nfields, P, S, done, tw, Wt, s);
}

hipError_t ns_finish(int nfields, int ncols, const double* part, double vol, double tol, double fp_floor,
                     int max_iter, int fixed, int first, int* done, int* iters, int* iters_out, double* resid,
                     int* status, int* const* fstat, const NsPark& pk, hipStream_t s) {
  hipLaunchKernelGGL(k_ns_finish, dim3(nfields), dim3(256), 0, s, ncols, part, vol, tol, fp_floor, max_iter, fixed,
                     first, done, iters, iters_out, resid, status, fstat, pk);
  return hipGetLastError();
}

__global__ void k_fill_int(int* p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t fill_int(int* p, int n, int v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_int, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

template <typename T>
static hipError_t cqcol(int ny, int nx, int nfields, const void* XH, double* part, double kx0, double ky0,
                        const void* tw, int Wt, hipStream_t s) {
  bool ok = false;
  dispatch_n(ny, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    ok = dispatch_w<T, N>(Wt, [&](auto wc) {
    constexpr int WT = decltype(wc)::value;
    using G = ColGeom<T, N, WT>;
    const int tiles = (nx / 2 + 1 + WT - 1) / WT;
    allow_lds(k_ns_cq_col<T, N, WT>, G::LDS_BYTES);
    hipLaunchKernelGGL((k_ns_cq_col<T, N, WT>), dim3(tiles * nfields), dim3(G::THREADS), G::LDS_BYTES, s,
                       (const cpx<T>*)XH, part, nx, tiles, kx0, ky0, (const cpx<T>*)tw);
    });
  });
  return ok ? hipGetLastError() : hipErrorInvalidValue;
}

hipError_t ns_cq_col(Prec p, int ny, int nx, int nfields, const void* XH, double* part, double kx0, double ky0,
                     const void* tw, int Wt, hipStream_t s) {
  return p == P32 ? cqcol<float>(ny, nx, nfields, XH, part, kx0, ky0, tw, Wt, s)
                  : cqcol<double>(ny, nx, nfields, XH, part, kx0, ky0, tw, Wt, s);
}

hipError_t ns_cq_finish(int nfields, int ncols, const double* part, double en_coef, double zz_coef, double* out,
                        int* status, hipStream_t s) {
  hipLaunchKernelGGL(k_ns_cq_finish, dim3(nfields), dim3(256), 0, s, ncols, part, en_coef, zz_coef, out, status);
  return hipGetLastError();
}

}  // namespace pst
