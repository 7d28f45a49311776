// Register/LDS Stockham FFT of one line, executed cooperatively by the
// N/R threads that own it (gfx950, wave64).
//
// Layout.  Thread t (0 <= t < N/R) of a line owns R complex values
// v[s] = x[t + s*(N/R)], s = 0..R-1.  Every stage reads its butterfly
// inputs from exactly these positions, so the first stage loads straight
// from global memory with unit stride across the wave, and after the last
// stage v[s] holds X[t + s*(N/R)] in natural order, stored back the same
// way.  Between stages the outputs go through LDS (Stockham autosort: a
// radix-r butterfly j with k = j mod Ns writes its outputs to
// (j/Ns)*Ns*r + k + q*Ns).  N = f * R^m with the odd-sized radix f (if any)
// first; a stage of radix r < R runs R/r butterflies per thread.
//
// Twiddles of stage s (radix r, Ns = product of earlier radices) come from
// a table of (r-1)*Ns entries, entry (q-1)*Ns + k = exp(-2 pi i q k /
// (Ns r)), computed in double precision on the host and rounded once.
// Single precision reads every entry it uses; double-precision radix-16
// stages read three entries per butterfly and form the other powers (see
// derived_twiddles).  The inverse transform multiplies by their conjugates.
// Transforms are unnormalised: forward kernel exp(-i...), inverse exp(+i...).
//
// The radix R of the full stages is a template parameter: 16 by default,
// or 8 (lines of 64 and more), which halves the values a thread must hold
// for one butterfly at the cost of one more exchange.  A length's table
// holds the radix-16 layout followed by the radix-8 one.
#pragma once

#include <type_traits>

#include "pst_common.hpp"

namespace pst {

// ---------------------------------------------------------------- stages ---
__host__ __device__ constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n / 2); }

__host__ __device__ constexpr int line_radix(int N) { return N < 16 ? N : 16; }

// Radix of the first stage (the leftover factor, or R if N is a power of R).
__host__ __device__ constexpr int first_radix(int N, int R) {
  return (ilog2c(N) % ilog2c(R)) == 0 ? R : (1 << (ilog2c(N) % ilog2c(R)));
}
__host__ __device__ constexpr int num_stages(int N, int R) {
  return (ilog2c(N) + ilog2c(R) - 1) / ilog2c(R);
}
__host__ __device__ constexpr int stage_radix(int N, int R, int s) {
  return s == 0 ? first_radix(N, R) : R;
}
__host__ __device__ constexpr int stage_ns(int N, int R, int s) {
  int ns = 1;
  for (int i = 0; i < s; ++i) ns *= stage_radix(N, R, i);
  return ns;
}
// Offset of stage s's twiddles in the per-length table.
__host__ __device__ constexpr int stage_tw_offset(int N, int R, int s) {
  int off = 0;
  for (int i = 1; i < s; ++i) off += (stage_radix(N, R, i) - 1) * stage_ns(N, R, i);
  return off;
}
__host__ __device__ constexpr int twiddle_table_len(int N, int R) {
  return stage_tw_offset(N, R, num_stages(N, R));
}
__host__ __device__ constexpr int twiddle_table_len(int N) { return twiddle_table_len(N, line_radix(N)); }
// Lengths that carry the radix-8 layout as well.
__host__ __device__ constexpr bool has_radix8(int N) { return N >= 64; }
// Entries of a length's table, and where the layout of radix R starts.
__host__ __device__ constexpr int tw_table_total(int N) {
  return twiddle_table_len(N) + (has_radix8(N) ? twiddle_table_len(N, 8) : 0);
}
__host__ __device__ constexpr int tw_base(int N, int R) { return R == line_radix(N) ? 0 : twiddle_table_len(N); }

// LDS slot of element e of a line: one pad slot every 16 elements.  A
// column tile interleaves its WS lines (slot * WS + line), so the lanes of a
// wave, which run over adjacent lines first, touch adjacent slots.
__host__ __device__ constexpr int lds_line_len(int N) { return N + N / 16; }
__host__ __device__ __forceinline__ int lds_idx(int e) { return e + (e >> 4); }

// ----------------------------------------------------------- butterflies ---
// Multiply by exp(-+ 2 pi i m / 16) with compile-time m; INV selects +.
//
// Single precision writes the rotation as v + v*(w - 1) with w in the first
// octant (angle pi/8 or pi/4) and the remaining multiple of pi/2 applied as
// an exact quarter turn.  The float pair (cos - 1, sin) below was chosen so
// that |w|^2 differs from 1 by ~1e-9 (the nearest floats of cos and sin give
// ~5e-8), so repeated transforms do not shrink or grow the field's norm.
struct Oct16f {
  static constexpr float A1 = -0x1.37ca18p-4f;  // cos(pi/8) - 1
  static constexpr float S1 = 0x1.87de2ap-2f;   // sin(pi/8)
  static constexpr float A2 = -0x1.2bec32p-2f;  // cos(pi/4) - 1
  static constexpr float S2 = 0x1.6a09e6p-1f;   // sin(pi/4)
};

// v * (1 + a + i s)
__host__ __device__ __forceinline__ cpx<float> rot_near1(cpx<float> v, float a, float s) {
  return cpx<float>{v.re + (v.re * a - v.im * s), v.im + (v.im * a + v.re * s)};
}

// v * (-i)^q (forward) or v * i^q (inverse)
template <bool INV, int Q, typename T>
__host__ __device__ __forceinline__ cpx<T> quarter(cpx<T> a) {
  constexpr int q = ((INV ? -Q : Q) % 4 + 4) % 4;  // number of -i factors
  if constexpr (q == 0) return a;
  else if constexpr (q == 1) return cpx<T>{a.im, -a.re};
  else if constexpr (q == 2) return cpx<T>{-a.re, -a.im};
  else return cpx<T>{-a.im, a.re};
}

template <bool INV, int M, typename T>
__host__ __device__ __forceinline__ cpx<T> rot16(cpx<T> a) {
  constexpr int m = ((M % 16) + 16) % 16;
  if constexpr (std::is_same<T, float>::value) {
    constexpr int r = m & 3;
    // forward W^m = exp(-2 pi i m/16): sign of the first-octant angle's sine
    constexpr float sg = INV ? 1.0f : -1.0f;
    if constexpr (r == 0) {
      return quarter<INV, m / 4>(a);
    } else if constexpr (r == 1) {
      return quarter<INV, m / 4>(rot_near1(a, Oct16f::A1, sg * Oct16f::S1));
    } else if constexpr (r == 2) {
      return quarter<INV, m / 4>(rot_near1(a, Oct16f::A2, sg * Oct16f::S2));
    } else {
      // W^m = W^{4(q+1)} W^{-1}
      return quarter<INV, m / 4 + 1>(rot_near1(a, Oct16f::A1, -sg * Oct16f::S1));
    }
  } else {
    if constexpr (m % 4 == 0) {
      return quarter<INV, m / 4>(a);
    } else {
      const T c = (T)cos16(m);
      const T s = INV ? (T)sin16(m) : -(T)sin16(m);
      return cpx<T>{a.re * c - a.im * s, a.re * s + a.im * c};
    }
  }
}

template <bool INV, typename T>
__host__ __device__ __forceinline__ void dft2(cpx<T>& a, cpx<T>& b) {
  cpx<T> t = a;
  a = t + b;
  b = t - b;
}

// In place: v[0..3] -> X[0..3].
template <bool INV, typename T>
__host__ __device__ __forceinline__ void dft4(cpx<T>& x0, cpx<T>& x1, cpx<T>& x2, cpx<T>& x3) {
  cpx<T> a0 = x0 + x2, a1 = x0 - x2, a2 = x1 + x3, a3 = x1 - x3;
  // forward: X1 = a1 - i a3, X3 = a1 + i a3
  cpx<T> ia3 = cpx<T>{-a3.im, a3.re};
  x0 = a0 + a2;
  x2 = a0 - a2;
  if (INV) {
    x1 = a1 + ia3;
    x3 = a1 - ia3;
  } else {
    x1 = a1 - ia3;
    x3 = a1 + ia3;
  }
}

template <bool INV, typename T>
__host__ __device__ __forceinline__ void dft8(cpx<T>* v) {
  // even/odd split: E = DFT4(x0,x2,x4,x6), O = DFT4(x1,x3,x5,x7)
  dft4<INV>(v[0], v[2], v[4], v[6]);
  dft4<INV>(v[1], v[3], v[5], v[7]);
  cpx<T> o1 = rot16<INV, 2>(v[3]), o2 = rot16<INV, 4>(v[5]), o3 = rot16<INV, 6>(v[7]);
  cpx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6], o0 = v[1];
  v[0] = e0 + o0; v[4] = e0 - o0;
  v[1] = e1 + o1; v[5] = e1 - o1;
  v[2] = e2 + o2; v[6] = e2 - o2;
  v[3] = e3 + o3; v[7] = e3 - o3;
}

template <bool INV, typename T>
__host__ __device__ __forceinline__ void dft16(cpx<T>* v) {
  // n = 4 n1 + n2, k = k1 + 4 k2:  DFT4 over n1, twiddle W16^(n2 k1), DFT4 over n2.
  dft4<INV>(v[0], v[4], v[8], v[12]);
  dft4<INV>(v[1], v[5], v[9], v[13]);
  dft4<INV>(v[2], v[6], v[10], v[14]);
  dft4<INV>(v[3], v[7], v[11], v[15]);
  // now v[n2 + 4 k1] = Y[n2][k1]
  v[5] = rot16<INV, 1>(v[5]);
  v[9] = rot16<INV, 2>(v[9]);
  v[13] = rot16<INV, 3>(v[13]);
  v[6] = rot16<INV, 2>(v[6]);
  v[10] = rot16<INV, 4>(v[10]);
  v[14] = rot16<INV, 6>(v[14]);
  v[7] = rot16<INV, 3>(v[7]);
  v[11] = rot16<INV, 6>(v[11]);
  v[15] = rot16<INV, 9>(v[15]);
  dft4<INV>(v[0], v[1], v[2], v[3]);
  dft4<INV>(v[4], v[5], v[6], v[7]);
  dft4<INV>(v[8], v[9], v[10], v[11]);
  dft4<INV>(v[12], v[13], v[14], v[15]);
  // v[n2 + 4 k1] now holds X[k1 + 4 n2]: transpose the 4x4 index grid.
  cpx<T> t;
  t = v[1]; v[1] = v[4]; v[4] = t;
  t = v[2]; v[2] = v[8]; v[8] = t;
  t = v[3]; v[3] = v[12]; v[12] = t;
  t = v[6]; v[6] = v[9]; v[9] = t;
  t = v[7]; v[7] = v[13]; v[13] = t;
  t = v[11]; v[11] = v[14]; v[14] = t;
}

template <int r, bool INV, typename T>
__host__ __device__ __forceinline__ void dft(cpx<T>* v) {
  if constexpr (r == 2) {
    dft2<INV>(v[0], v[1]);
  } else if constexpr (r == 4) {
    dft4<INV>(v[0], v[1], v[2], v[3]);
  } else if constexpr (r == 8) {
    dft8<INV>(v);
  } else if constexpr (r == 16) {
    dft16<INV>(v);
  }
}

// ------------------------------------------------------------ line FFT ---
// LDS addressing with one base per butterfly and compile-time offsets: for
// every stage shape used here (Ns a power of two; Ns >= 16, or base mod 16 <
// Ns with q*Ns mod 16 <= 16 - Ns, or Ns = 1 with base a multiple of the
// radix), lds_idx(base + q*Ns) = lds_idx(base) + q*Ns + ((q*Ns) >> 4), and
// lds_idx(t + s*TL) = lds_idx(t) + s*TL + ((s*TL) >> 4) for t < TL.
__host__ __device__ constexpr int lds_off(int x) { return x + (x >> 4); }

// Twiddle load: entry `idx` of a line length's table of `len` entries.  On
// the device it goes through a buffer resource with the stage/radix part of
// the index as a wave-uniform scalar offset, so a thread's twiddle
// addresses cost one register per stage instead of a 64-bit address per
// entry (which the compiler would otherwise keep live across every
// transform of a kernel).
template <typename T>
__host__ __device__ __forceinline__ cpx<T> tw_load(const cpx<T>* tw, int len, unsigned k, unsigned base) {
#if defined(__HIP_DEVICE_COMPILE__)
  const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<cpx<T>*>(tw), 0, len * (int)sizeof(cpx<T>), 0x00020000);
  if constexpr (sizeof(T) == 4) {
    using V = float __attribute__((ext_vector_type(2)));
    const V a = __builtin_bit_cast(
        V, __builtin_amdgcn_raw_buffer_load_b64(r, k * (unsigned)sizeof(cpx<T>), base * (unsigned)sizeof(cpx<T>), 0));
    return {a.x, a.y};
  } else {
    using V = double __attribute__((ext_vector_type(2)));
    const V a = __builtin_bit_cast(
        V, __builtin_amdgcn_raw_buffer_load_b128(r, k * (unsigned)sizeof(cpx<T>), base * (unsigned)sizeof(cpx<T>), 0));
    return {a.x, a.y};
  }
#else
  (void)len;
  return tw[base + k];
#endif
}

// Double-precision radix-16 stages after the first read three table
// entries per butterfly, the powers 1, 4 and 8 of its base twiddle
// c = exp(-2 pi i k / (16 Ns)), and form the other twelve powers by complex
// products (c^15 = c^8 (c^4 (c^2 c)) is four products deep: a few units of
// 2^-53): fifteen table loads per butterfly cost more time than the
// products.  These loads are issued before the preceding exchange, so their
// latency hides behind it.  Single precision reads all fifteen entries:
// each is the float pair of modulus closest to 1 near the exact value, and
// products of such pairs would lose that.
template <typename T>
__host__ __device__ constexpr bool derived_twiddles(int r) {
  return r == 16 && std::is_same<T, double>::value;
}

// c^1, c^4 and c^8 for butterfly j of stage S.
template <int N, int S, int R, typename T>
__host__ __device__ __forceinline__ void load_roots(cpx<T> (&c)[3], const cpx<T>* __restrict__ tw, int j) {
  constexpr int Ns = stage_ns(N, R, S);
  constexpr int toff = tw_base(N, R) + stage_tw_offset(N, R, S);
  const unsigned k = (unsigned)j & (Ns - 1);
  c[0] = tw_load(tw, tw_table_total(N), k, (unsigned)toff);
  c[1] = tw_load(tw, tw_table_total(N), k, (unsigned)(toff + 3 * Ns));
  c[2] = tw_load(tw, tw_table_total(N), k, (unsigned)(toff + 7 * Ns));
}

// w[q] *= c^q (forward) or conj(c)^q (inverse), q = 1..15, from c^1, c^4, c^8.
template <bool INV, typename T>
__host__ __device__ __forceinline__ void apply_powers(cpx<T>* w, cpx<T> c1, cpx<T> c4, cpx<T> c8) {
  cpx<T> c[16];
  c[1] = c1;
  c[4] = c4;
  c[8] = c8;
  c[2] = cmul(c[1], c[1]);
  c[3] = cmul(c[2], c[1]);
  c[5] = cmul(c[4], c[1]);
  c[6] = cmul(c[4], c[2]);
  c[7] = cmul(c[4], c[3]);
#pragma unroll
  for (int q = 9; q < 16; ++q) c[q] = cmul(c[8], c[q - 8]);
#pragma unroll
  for (int q = 1; q < 16; ++q) w[q] = INV ? cmul_conj(w[q], c[q]) : cmul(w[q], c[q]);
}

// Base twiddles of one derived-twiddle stage for a thread's butterflies,
// loaded while the previous stage's exchange is in progress.
template <int VPT, int R, typename T>
struct NextRoots {
  cpx<T> c[VPT / R > 0 ? VPT / R : 1][3];
};

// One Stockham stage for thread t.  A thread owns VPT values (VPT a
// multiple of every stage radix; TL = N/VPT threads per line) and runs VPT/r
// butterflies of the stage; outputs either stay in registers (last stage) or
// go to the line's LDS slots.  SPLIT exchanges real parts, then imaginary
// parts, through a buffer of scalars (half the LDS); the imaginary outputs
// wait in the consumed input registers meanwhile.
template <int N, int S, bool INV, int WS, int VPT, bool SPLIT, int R, typename T>
__host__ __device__ __forceinline__ void line_stage(cpx<T> (&v)[VPT], void* ldsv, int t,
                                                    const cpx<T>* __restrict__ tw,
                                                    const NextRoots<VPT, R, T>& pre) {
  static_assert(R == line_radix(N) || (R == 8 && has_radix8(N)), "no twiddle layout for this radix");
  constexpr int TL = N / VPT;
  constexpr int r = stage_radix(N, R, S);
  constexpr int Ns = stage_ns(N, R, S);
  constexpr int B = VPT / r;
  constexpr bool last = (S == num_stages(N, R) - 1);
  constexpr int toff = tw_base(N, R) + stage_tw_offset(N, R, S);
  static_assert(VPT % r == 0, "values per thread must be a multiple of each radix");
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int j = t + b * TL;
    cpx<T> w[r];
#pragma unroll
    for (int q = 0; q < r; ++q) w[q] = v[b + q * B];
    if constexpr (Ns > 1) {
      if constexpr (derived_twiddles<T>(r)) {
        apply_powers<INV>(w, pre.c[b][0], pre.c[b][1], pre.c[b][2]);
      } else {
        const unsigned k = (unsigned)j & (Ns - 1);
#pragma unroll
        for (int q = 1; q < r; ++q) {
          // uniform base toff + (q-1) Ns, per-lane offset k
          const cpx<T> c = tw_load(tw, tw_table_total(N), k, (unsigned)(toff + (q - 1) * Ns));
          w[q] = INV ? cmul_conj(w[q], c) : cmul(w[q], c);
        }
      }
    }
    dft<r, INV>(w);
    if constexpr (last) {
#pragma unroll
      for (int q = 0; q < r; ++q) v[b + q * B] = w[q];
    } else {
      const int base = ((j / Ns) * Ns * r) + (j & (Ns - 1));
      if constexpr (SPLIT) {
        T* pw = static_cast<T*>(ldsv) + lds_idx(base) * WS;
#pragma unroll
        for (int q = 0; q < r; ++q) {
          pw[lds_off(q * Ns) * WS] = w[q].re;
          v[b + q * B].im = w[q].im;
        }
      } else {
        cpx<T>* pw = static_cast<cpx<T>*>(ldsv) + lds_idx(base) * WS;
#pragma unroll
        for (int q = 0; q < r; ++q) pw[lds_off(q * Ns) * WS] = w[q];
      }
    }
  }
}

// Second half of a split exchange: the imaginary outputs parked in v[].im go
// to the same slots the real parts used.
template <int N, int S, int WS, int VPT, int R, typename T>
__host__ __device__ __forceinline__ void line_stage_im(const cpx<T> (&v)[VPT], T* lds, int t) {
  constexpr int TL = N / VPT;
  constexpr int r = stage_radix(N, R, S);
  constexpr int Ns = stage_ns(N, R, S);
  constexpr int B = VPT / r;
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int j = t + b * TL;
    const int base = ((j / Ns) * Ns * r) + (j & (Ns - 1));
    T* pw = lds + lds_idx(base) * WS;
#pragma unroll
    for (int q = 0; q < r; ++q) pw[lds_off(q * Ns) * WS] = v[b + q * B].im;
  }
}

template <int N, int WS, int VPT, typename T>
__host__ __device__ __forceinline__ void line_read(cpx<T> (&v)[VPT], const cpx<T>* lds, int t) {
  constexpr int TL = N / VPT;
  const cpx<T>* pr = lds + lds_idx(t) * WS;
#pragma unroll
  for (int s = 0; s < VPT; ++s) v[s] = pr[lds_off(s * TL) * WS];
}

template <int N, int WS, int VPT, bool IM, typename T>
__host__ __device__ __forceinline__ void line_read_part(cpx<T> (&v)[VPT], const T* lds, int t) {
  constexpr int TL = N / VPT;
  const T* pr = lds + lds_idx(t) * WS;
#pragma unroll
  for (int s = 0; s < VPT; ++s) {
    if constexpr (IM) v[s].im = pr[lds_off(s * TL) * WS];
    else v[s].re = pr[lds_off(s * TL) * WS];
  }
}

template <int N, int S, bool INV, int WS, int VPT, bool SPLIT, int R, typename T>
__device__ __forceinline__ void line_stages(cpx<T> (&v)[VPT], void* lds, int t, const cpx<T>* __restrict__ tw,
                                            const NextRoots<VPT, R, T>& pre) {
  if constexpr (S < num_stages(N, R)) {
    line_stage<N, S, INV, WS, VPT, SPLIT, R>(v, lds, t, tw, pre);
    if constexpr (S < num_stages(N, R) - 1) {
      // the next stage's base twiddles are in flight during the exchange
      NextRoots<VPT, R, T> nxt;
      if constexpr (derived_twiddles<T>(R)) {
        constexpr int TL = N / VPT;
#pragma unroll
        for (int b = 0; b < VPT / R; ++b) load_roots<N, S + 1, R>(nxt.c[b], tw, t + b * TL);
      }
      __syncthreads();
      if constexpr (SPLIT) {
        line_read_part<N, WS, VPT, false>(v, static_cast<const T*>(lds), t);
        __syncthreads();
        line_stage_im<N, S, WS, VPT, R>(v, static_cast<T*>(lds), t);
        __syncthreads();
        line_read_part<N, WS, VPT, true>(v, static_cast<const T*>(lds), t);
      } else {
        line_read<N, WS, VPT>(v, static_cast<const cpx<T>*>(lds), t);
      }
      __syncthreads();
      line_stages<N, S + 1, INV, WS, VPT, SPLIT, R>(v, lds, t, tw, nxt);
    }
  }
}

// Full unnormalised FFT of a line whose N/VPT owners all call this together
// (every thread of the block must call it: it contains block barriers).
// lds points at the line's first slot (complex, or scalar when SPLIT); WS is
// the slot stride (lines per interleaved tile).
template <int N, bool INV, int WS = 1, int VPT = line_radix(N), bool SPLIT = false, int R = line_radix(N),
          typename T>
__device__ __forceinline__ void line_fft(cpx<T> (&v)[VPT], void* lds, int t, const cpx<T>* __restrict__ tw) {
  line_stages<N, 0, INV, WS, VPT, SPLIT, R>(v, lds, t, tw, NextRoots<VPT, R, T>{});
}

}  // namespace pst
