// Pass geometry and shared helpers of the pst kernels (gfx950).
//
// A "row pass" transforms lines along x (contiguous, length nx); a "column
// pass" transforms lines along y (stride = row length, length ny).  Both
// keep a line in registers (R values per thread, N/R threads per line) and
// use LDS only for the exchanges between Stockham stages.
#pragma once

#include <type_traits>
#include <utility>

#include "fft_line.hpp"
#include "launch.hpp"

namespace pst {

// LDS slots per line, including one pad slot per 16 elements and a tail
// that shifts consecutive lines of a column tile by half of the LDS bank
// space (128 bytes).
template <typename T>
__host__ __device__ constexpr int lds_line_stride(int N) {
  return N + N / 16 + (int)(128 / sizeof(cpx<T>));
}

// Row pass: LPB lines per block, N/VPT threads per line, >= 256 threads
// per block when the line is short.  SPLIT exchanges real and imaginary
// parts one after the other through half the LDS.
template <typename T, int N, int VPT = line_radix(N), bool SPLIT = false>
struct RowGeom {
  static constexpr int R = VPT;
  static constexpr int TL = N / VPT;
  static constexpr int LPB = TL >= 256 ? 1 : 256 / TL;
  static constexpr int THREADS = LPB * TL;
  static constexpr int STRIDE = SPLIT ? N + N / 16 + (int)(128 / sizeof(T)) : lds_line_stride<T>(N);
  static constexpr size_t LDS_BYTES = (size_t)LPB * STRIDE * (SPLIT ? sizeof(T) : sizeof(cpx<T>));
};

// Column pass: W adjacent columns per block, thread (c, t) with c fastest so
// that a wave reads W consecutive elements of a row per instruction; the W
// lines are interleaved in LDS (slot * W + c).  VPT values per thread
// (N/VPT threads per line); SPLIT exchanges real and imaginary parts one
// after the other through half the LDS.
template <typename T, int N, int W, int VPT = line_radix(N), bool SPLIT = false>
struct ColGeom {
  static constexpr int R = VPT;
  static constexpr int TL = N / VPT;
  static constexpr int THREADS = W * TL;
  static constexpr size_t LDS_BYTES = (size_t)W * lds_line_len(N) * (SPLIT ? sizeof(T) : sizeof(cpx<T>));
};

// Column tile variants compiled for a column length (the autotuner picks
// one per plan).  Variant 0: the largest W with W*N/16 <= 1024 threads,
// W <= 16 and <= 150 KB of LDS, 16 values per thread, complex exchange.
// Single-field passes (NLS, C2C) of FP32 lines of 4096 and more, whose
// variant-0 block fills a CU alone, add variants that let two blocks share
// a CU or widen the row segments: 1, the same W with 32 values per thread
// and the split exchange (half the threads and half the LDS); 2, the same W
// with 16 values per thread, the split exchange and registers capped for 8
// waves per SIMD; 3, twice the W with 32 values per thread and the split
// exchange (variant 0's threads and LDS); 4, variant 2 without the register
// cap.  Otherwise variant 1 is half of variant 0's W, and single-field FP64
// passes of 4096 and more add 2, variant 0's W with 32 values per thread
// and the split exchange (registers capped for 2 waves per SIMD); 3, variant
// 0's W with the split exchange and registers capped for 4 waves per SIMD
// (two blocks per CU); 4, twice that W (full
// 128-byte row segments, one 1024-thread block per CU); 5, variant 0's W at
// radix 8 (8 values per thread, twice the threads) with the split exchange.
template <typename T, int N>
struct ColTiles {
  static constexpr int TL = N / line_radix(N);
  static constexpr int fit(int w) {
    return (w * TL <= 1024 && (size_t)w * lds_line_len(N) * sizeof(cpx<T>) <= 150 * 1024) ? w : 0;
  }
  static constexpr int WMAX = fit(16) ? 16 : fit(8) ? 8 : fit(4) ? 4 : fit(2) ? 2 : 1;
  static constexpr int WALT = WMAX > 1 ? WMAX / 2 : 1;
  static constexpr bool SPLIT1 = std::is_same<T, float>::value && N >= 4096;
  static constexpr bool SPLIT2 = std::is_same<T, double>::value && N >= 4096;
};

// W columns per block, VPT values per thread, split exchange, the minimum
// waves per SIMD the register allocation must allow (1: no cap), radix of
// the full stages.
template <int W, int VPT, bool SPLIT, int WPE = 1, int R = 16>
struct ColCfg {
  static constexpr int w = W, vpt = VPT, wpe = WPE, radix = R;
  static constexpr bool split = SPLIT;
};

// Calls f(ColCfg<...>) for variant `var` of a single-field column pass.
template <typename T, int N, class F>
bool dispatch_col1(int var, F&& f) {
  using CT = ColTiles<T, N>;
  constexpr int R = line_radix(N);
  if (var == 0) {
    f(ColCfg<CT::WMAX, R, false, 1, R>{});
    return true;
  }
  if constexpr (CT::SPLIT1) {
    if (var == 1) {
      f(ColCfg<CT::WMAX, 32, true>{});
      return true;
    }
    if (var == 2) {
      f(ColCfg<CT::WMAX, R, true, 8>{});
      return true;
    }
    if (var == 3) {
      f(ColCfg<2 * CT::WMAX, 32, true>{});
      return true;
    }
    if (var == 4) {
      f(ColCfg<CT::WMAX, R, true>{});
      return true;
    }
  } else if (var == 1) {
    f(ColCfg<CT::WALT, R, false, 1, R>{});
    return true;
  }
  if constexpr (CT::SPLIT2) {
    if (var == 2) {
      f(ColCfg<CT::WMAX, 32, true, 2>{});
      return true;
    }
    if (var == 3) {
      f(ColCfg<CT::WMAX, 16, true, 4>{});
      return true;
    }
    if (var == 4) {
      f(ColCfg<2 * CT::WMAX, 16, true>{});
      return true;
    }
    if (var == 5) {
      f(ColCfg<CT::WMAX, 8, true, 1, 8>{});
      return true;
    }
  }
  return false;
}

// Row variants of the NLS in-place row pass (the pass that runs every step),
// for lines of length N.  Lines of 4096 and more run one line per block:
// 0, 16 values per thread and the complex exchange (32 values and the split
// exchange at 8192); 1, 16 values and the split exchange (half the LDS);
// 2, radix 8 with 8 values per thread (twice the threads, fewer registers)
// and the split exchange; 3, radix 8 with the complex exchange.  Shorter
// lines run row pairs, P pairs per block: 0, the default P (256 threads);
// then half of it (where P >= 2) and twice it (where that fits 1024 threads
// and 150 KB of LDS), numbered in that order.  P = 0 in a config means the
// default.
template <int VPT, bool SPLIT, int R, int P>
struct RowCfg {
  static constexpr int vpt = VPT, radix = R, pairs = P;
  static constexpr bool split = SPLIT;
};
template <int N>
struct NlsRowShape {
  static constexpr bool ONE_LINE = N / line_radix(N) >= 256;  // one line per block
  static constexpr int TL = N / line_radix(N);
  static constexpr int P0 = TL >= 128 ? 1 : 128 / TL;          // default pairs per block
};
template <typename T, int N, class F>
bool dispatch_nls_row(int var, F&& f) {
  using S = NlsRowShape<N>;
  constexpr int R = line_radix(N);
  if constexpr (S::ONE_LINE) {
    if (var == 0) {
      if constexpr (N >= 8192) f(RowCfg<32, true, 16, 0>{});
      else f(RowCfg<16, false, 16, 0>{});
      return true;
    }
    if (var == 1) {
      f(RowCfg<16, true, 16, 0>{});
      return true;
    }
    if (var == 2) {
      f(RowCfg<8, true, 8, 0>{});
      return true;
    }
    if (var == 3) {
      f(RowCfg<8, false, 8, 0>{});
      return true;
    }
  } else {
    if (var == 0) {
      f(RowCfg<R, false, R, 0>{});
      return true;
    }
    // the others are numbered in order of those that exist
    int k = 1;
    if constexpr (S::P0 >= 2) {
      if (var == k) {
        f(RowCfg<R, false, R, S::P0 / 2>{});
        return true;
      }
      ++k;
    }
    constexpr size_t lds2 = (size_t)4 * S::P0 * lds_line_len(N) * sizeof(cpx<T>);
    if constexpr (4 * S::P0 * S::TL <= 1024 && lds2 <= 150 * 1024) {
      if (var == k) {
        f(RowCfg<R, false, R, 2 * S::P0>{});
        return true;
      }
    }
  }
  return false;
}

// Calls f(IntC<W>) for variant `var` of a two-line column pass.
template <typename T, int N, class F>
// Lines of 512 and more add a quarter and an eighth of variant 0's W (as
// far as they are >= 1): a batch of small fields then runs several blocks
// per CU instead of one.
bool dispatch_w(int var, F&& f) {
  using CT = ColTiles<T, N>;
  if (var == 0) {
    f(std::integral_constant<int, CT::WMAX>{});
    return true;
  }
  if (var == 1) {
    f(std::integral_constant<int, CT::WALT>{});
    return true;
  }
  if constexpr (N >= 512 && CT::WMAX >= 4) {
    if (var == 2) {
      f(std::integral_constant<int, CT::WMAX / 4>{});
      return true;
    }
  }
  if constexpr (N >= 512 && CT::WMAX >= 8) {
    if (var == 3) {
      f(std::integral_constant<int, CT::WMAX / 8>{});
      return true;
    }
  }
  return false;
}

// Pointer into the global address space.  Fields reached through a
// FieldRef (base + stride or a device pointer table) are plain pointers to
// the compiler; accessing them through gptr makes it emit global (not flat)
// memory instructions, which do not share the LDS wait counter.
template <typename P>
using gptr = __attribute__((address_space(1))) P*;
template <typename P>
__device__ __forceinline__ gptr<P> field(const FieldRef& f, int i) {
  return (gptr<P>)f.at(i);
}
// Stores write at most 8 bytes per lane.  On gfx950 a vector memory store
// of 16 bytes whose data registers the next VALU instruction overwrites can
// write the new values (observed as run-to-run differences in FP64 results:
// the compiler put no wait state between the two), so 16-byte values go out
// as two 8-byte halves, and every store made through these helpers uses an
// address the compiler cannot relate to its neighbours', so that it does not
// merge adjacent stores back into one wide access.
template <typename P>
__device__ __forceinline__ gptr<P> unmerged(gptr<P> p) {
  asm volatile("" : "+v"(p));
  return p;
}
template <typename T>
__device__ __forceinline__ void store1(gptr<T> p, T v) {
  static_assert(sizeof(T) <= 8, "stores write at most 8 bytes");
  *unmerged(p) = v;
}
template <typename T>
__device__ __forceinline__ void store1(T* p, T v) {
  store1((gptr<T>)p, v);
}

// Load and store of a complex value through a global pointer (one 8- or
// 16-byte load; one or two 8-byte stores).
template <typename T>
__device__ __forceinline__ cpx<T> gload(gptr<const cpx<T>> p) {
  using V = T __attribute__((ext_vector_type(2)));
  const V a = *(gptr<const V>)p;
  return {a.x, a.y};
}
template <typename T>
__device__ __forceinline__ cpx<T> gload(gptr<cpx<T>> p) {
  return gload((gptr<const cpx<T>>)p);
}
template <typename T>
__device__ __forceinline__ void gstore(gptr<cpx<T>> p, cpx<T> v) {
  if constexpr (sizeof(T) == 4) {
    using V = T __attribute__((ext_vector_type(2)));
    store1((gptr<V>)p, V{v.re, v.im});
  } else {
    store1((gptr<T>)p, v.re);
    store1((gptr<T>)p + 1, v.im);
  }
}
template <typename T>
__device__ __forceinline__ void gstore(cpx<T>* p, cpx<T> v) {
  gstore((gptr<cpx<T>>)p, v);
}

// Buffer-resource access to one field (at most 2 GiB): 32-bit byte offsets,
// a per-lane part (voff) and a wave-uniform part (soff, kept in a scalar
// register), so a thread's many strided accesses cost no 64-bit address
// registers.  Word 3 of the descriptor is the gfx9 raw-buffer format.
// 16-byte stores (an FP64 complex value, or two FP32 ones) are issued from
// an asm statement that ends with two wait states, so that no instruction
// can overwrite the data registers right behind the store (the hazard
// described above); the compiler sees the statement as a store to memory.
struct FieldBuf {
  __amdgpu_buffer_rsrc_t r;
  __device__ FieldBuf(const void* base, unsigned bytes)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, 0x00020000)) {}
  __device__ __forceinline__ cpx<float> ld(cpx<float>*, unsigned voff, unsigned soff) const {
    using V = float __attribute__((ext_vector_type(2)));
    const V a = __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    return {a.x, a.y};
  }
  __device__ __forceinline__ cpx<double> ld(cpx<double>*, unsigned voff, unsigned soff) const {
    using V = double __attribute__((ext_vector_type(2)));
    const V a = __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
    return {a.x, a.y};
  }
  __device__ __forceinline__ void st(unsigned voff, unsigned soff, cpx<float> v) const {
    using V = float __attribute__((ext_vector_type(2)));
    using U = unsigned long long __attribute__((ext_vector_type(1)));
    const V a = {v.re, v.im};
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U, a), r, voff, soff, 0);
  }
  __device__ __forceinline__ void st16(unsigned voff, unsigned soff,
                                       unsigned __attribute__((ext_vector_type(4))) data) const {
    asm volatile("buffer_store_dwordx4 %0, %1, %2, %3 offen\n\ts_nop 1"
                 :
                 : "v"(data), "v"(voff), "s"(r), "s"(soff)
                 : "memory");
  }
  __device__ __forceinline__ void st(unsigned voff, unsigned soff, cpx<double> v) const {
    using V = double __attribute__((ext_vector_type(2)));
    using U = unsigned __attribute__((ext_vector_type(4)));
    st16(voff, soff, __builtin_bit_cast(U, V{v.re, v.im}));
  }
  template <typename T>
  __device__ __forceinline__ cpx<T> ldc(unsigned voff, unsigned soff) const {
    return ld((cpx<T>*)nullptr, voff, soff);
  }
  // two adjacent complex values (one 16-byte access in FP32)
  __device__ __forceinline__ void ld2(unsigned voff, cpx<float>& a, cpx<float>& b) const {
    using V = float __attribute__((ext_vector_type(4)));
    const V x = __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(r, voff, 0, 0));
    a = {x.x, x.y};
    b = {x.z, x.w};
  }
  __device__ __forceinline__ void ld2(unsigned voff, cpx<double>& a, cpx<double>& b) const {
    a = ld((cpx<double>*)nullptr, voff, 0);
    b = ld((cpx<double>*)nullptr, voff, (unsigned)sizeof(cpx<double>));
  }
  __device__ __forceinline__ void st2(unsigned voff, cpx<float> a, cpx<float> b) const {
    using V = float __attribute__((ext_vector_type(4)));
    using U = unsigned __attribute__((ext_vector_type(4)));
    st16(voff, 0, __builtin_bit_cast(U, V{a.re, a.im, b.re, b.im}));
  }
  __device__ __forceinline__ void st2(unsigned voff, cpx<double> a, cpx<double> b) const {
    st(voff, 0, a);
    st(voff, (unsigned)sizeof(cpx<double>), b);
  }
};

// A column tile's view of one complex array laid out [field][N][ncols]:
// element s of thread (c, t) is row t + s*TL of column col of the block's
// field (field must be block-uniform).  IL: the rows of each pair (2p, 2p+1)
// are interleaved element by element, (y, x) at (y - y%2) ncols + 2x + y%2,
// so that W adjacent columns span 2W-element segments.  Columns past the
// end get an offset beyond the buffer's range, so their loads read zeros and
// their stores are dropped by the hardware range check.
template <typename T, bool IL = false>
struct ColArr {
  FieldBuf b;
  unsigned o0, ds;
  bool one;  // TL == 1 (interleaved lines of 16 or less): parity of y is that of s
  __device__ ColArr(const void* array, int field, int N, int ncols, int col, bool valid, int t, int TL)
      : b((const char*)array + (size_t)field * N * ncols * sizeof(cpx<T>),
          (unsigned)((size_t)N * ncols * sizeof(cpx<T>))),
        o0(!valid ? 0x80000000u
                  : (unsigned)(IL ? (t & ~1) * ncols + 2 * col + (t & 1) : col + t * ncols) *
                        (unsigned)sizeof(cpx<T>)),
        ds((unsigned)(TL * ncols) * (unsigned)sizeof(cpx<T>)),
        one(IL && TL == 1) {}
  // TL == 1: y = s, so an odd s is one element past o0 and one row short of s ds
  __device__ __forceinline__ unsigned voff(int s) const {
    return one && (s & 1) && o0 != 0x80000000u ? o0 + (unsigned)sizeof(cpx<T>) : o0;
  }
  __device__ __forceinline__ unsigned soff(int s) const { return one && (s & 1) ? (s - 1) * ds : s * ds; }
  __device__ __forceinline__ cpx<T> ld(int s) const { return b.template ldc<T>(voff(s), soff(s)); }
  __device__ __forceinline__ void st(int s, cpx<T> v) const { b.st(voff(s), soff(s), v); }
};

// Keeps the compiler from moving memory accesses across this point (used to
// stop loads for a later phase being hoisted above a transform, where they
// would hold registers through it).
__device__ __forceinline__ void mem_fence_compiler() { asm volatile("" ::: "memory"); }

// Blocks are handed to the 8 XCDs of the chip round robin (block b runs on
// XCD b mod 8).  Give each XCD a contiguous range of tiles, so that the
// column tiles sharing a 128-byte line are read through the same L2.
__device__ __forceinline__ int xcd_tile(int b, int nblocks) {
  const int q = nblocks >> 3, rem = nblocks & 7;
  const int x = b & 7, i = b >> 3;
  return x * q + (x < rem ? x : rem) + i;
}

// Single-precision sine and cosine with the argument reduced in double
// precision: n = nearest integer to x / (pi/2), r = x - n pi/2 (one double
// FMA, so |r| <= pi/4 to double accuracy for any |x| below ~1e15), then the
// Taylor series of sin and cos to degree 9 and 10 in r (truncation below
// 2e-9 on |r| <= pi/4, under FP32 rounding), and the quadrant n mod 4 picks
// +-sin r or +-cos r.  Compact (no large-argument branch), which keeps
// register use low when many values are evaluated at once.
__device__ __forceinline__ void sincos_f32(float x, float& sn, float& cs) {
  const double xd = x;
  const double n = rint(xd * 0.63661977236758134308);       // 2 / pi
  float r = (float)fma(-n, 1.57079632679489661923, xd);  // pi / 2
  // |x| beyond ~1e15 (where FP32 carries no phase information) gives a
  // bounded value; NaN and infinity propagate
  if (fabsf(r) > 0.8f) r = 0.0f;
  const double q4 = n - 4.0 * floor(n * 0.25);                 // n mod 4, exact
  const int q = (int)q4;
  const float r2 = r * r;
  // sin r = r (1 - r^2/3! + r^4/5! - r^6/7! + r^8/9!)
  const float ps = r * (1.0f + r2 * (-1.0f / 6 + r2 * (1.0f / 120 + r2 * (-1.0f / 5040 + r2 * (1.0f / 362880)))));
  // cos r = 1 - r^2/2! + r^4/4! - r^6/6! + r^8/8! - r^10/10!
  const float pc =
      1.0f + r2 * (-0.5f + r2 * (1.0f / 24 + r2 * (-1.0f / 720 + r2 * (1.0f / 40320 + r2 * (-1.0f / 3628800)))));
  const float s0 = (q & 1) ? pc : ps, c0 = (q & 1) ? ps : pc;
  sn = (q & 2) ? -s0 : s0;
  cs = ((q + 1) & 2) ? -c0 : c0;
}
__device__ __forceinline__ float sin_f32(float x) {
  float s, c;
  sincos_f32(x, s, c);
  return s;
}

// v * exp(-i theta), written as v + v*(cos(theta) - 1 - i sin(theta)) with
// cos(theta) - 1 = -2 sin^2(theta/2): for the small angles of a time step
// the correction is tiny, so rounding does not bias |v| (a rounded
// cos(theta) near 1 would).  Short Taylor series for small angles, the
// half angle's sine and cosine otherwise.
__device__ __forceinline__ cpx<float> rotate_neg(cpx<float> v, float th) {
  float cm1, s;
  if (fabsf(th) <= 0.03125f) {
    // |theta| <= 2^-5: truncation below 2e-12 (cos - 1) and 3e-10 (sin)
    const float t2 = th * th;
    cm1 = t2 * (-0.5f + t2 * (1.0f / 24));
    s = th * (1.0f - t2 * (1.0f / 6));
  } else {
    float sh, ch;
    sincos_f32(0.5f * th, sh, ch);
    cm1 = -2.0f * sh * sh;
    s = 2.0f * sh * ch;
  }
  return cpx<float>{v.re + (v.re * cm1 + v.im * s), v.im + (v.im * cm1 - v.re * s)};
}
__device__ __forceinline__ cpx<double> rotate_neg(cpx<double> v, double th) {
  double cm1, s;
  if (fabs(th) <= 0.03125) {
    // |theta| <= 2^-5: Taylor series of cos - 1 to theta^10 and of sin to
    // theta^11; the first omitted terms are below 2^-110 and 2^-104
    // relative to cos - 1 and sin (under double rounding), and the series
    // costs a dozen FMAs against the library routine's range reduction
    const double t2 = th * th;
    cm1 = t2 * (-0.5 + t2 * (1.0 / 24 + t2 * (-1.0 / 720 + t2 * (1.0 / 40320 + t2 * (-1.0 / 3628800)))));
    s = th * (1.0 + t2 * (-1.0 / 6 + t2 * (1.0 / 120 + t2 * (-1.0 / 5040 + t2 * (1.0 / 362880 + t2 * (-1.0 / 39916800))))));
  } else {
    double sh, ch;
    sincos(0.5 * th, &sh, &ch);
    cm1 = -2.0 * sh * sh;
    s = 2.0 * sh * ch;
  }
  return cpx<double>{v.re + (v.re * cm1 + v.im * s), v.im + (v.im * cm1 - v.re * s)};
}

// Deterministic sum of one double per thread over the n threads of a line
// (n a power of two); the thread with index t of line `line` owns slot
// line*n + t of red.  Tree order is fixed.  Every thread of the block must
// call it with the same n.  The result is returned to every thread of the
// line.
__device__ __forceinline__ double line_sum(double* red, int line, int t, int n, double v) {
  double* r = red + line * n;
  r[t] = v;
  __syncthreads();
  for (int h = n >> 1; h > 0; h >>= 1) {
    if (t < h) r[t] += r[t + h];
    __syncthreads();
  }
  const double out = r[0];
  __syncthreads();
  return out;
}

template <typename T>
__device__ __forceinline__ bool finite_c(cpx<T> v) {
  return isfinite(v.re) && isfinite(v.im);
}

// Latch ST_NONFINITE for field f when this thread saw a non-finite value.
// Only the first such lane of a wave writes when the whole wave works on
// field f (wave_uniform), so a field flooded with NaN costs one atomic per
// wave; otherwise every such lane writes its own field's word.
__device__ __forceinline__ void latch_nonfinite(bool bad, const StatusRef& st, int f, bool wave_uniform) {
  if (!bad) return;
  if (wave_uniform) {
    const unsigned long long m = __ballot(1);  // lanes with bad set (the others returned)
    if ((int)(__lane_id()) != __ffsll((long long)m) - 1) return;
  }
  if (st.plan != nullptr) atomicOr(st.plan, (int)ST_NONFINITE);
  if (st.field != nullptr && st.field[f] != nullptr) atomicOr(st.field[f], (int)ST_NONFINITE);
}

// Kernels whose dynamic LDS exceeds 64 KiB must opt in once (gfx950 has
// 160 KiB per workgroup).
template <class K>
inline void allow_lds(K kernel, size_t bytes) {
  if (bytes > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// ------------------------------------------------------ real row pairs ---
// Two real rows a, b travel as one complex line z = a + i b.


// After the forward transform Z of z = a + i b (natural order in v), store
// 2*A[k] = Z[k] + conj(Z[n-k]) and 2*B[k] = -i (Z[k] - conj(Z[n-k])) for
// k = 0..n/2 (the half spectra of rows a and b, times 2).  Uses the line's
// LDS buffer; contains block barriers, the last one after its LDS reads, so
// a transform may follow at once.
template <typename T, int N>
__device__ __forceinline__ void store_pair_halves(const cpx<T> (&v)[line_radix(N)], cpx<T>* L, int t,
                                                  cpx<T>* A, cpx<T>* B, bool va, bool vb) {
  constexpr int R = line_radix(N);
  constexpr int TL = N / R;
  __syncthreads();
#pragma unroll
  for (int s = 0; s < R; ++s) L[lds_idx(t + s * TL)] = v[s];
  __syncthreads();
#pragma unroll
  for (int s = 0; s <= R / 2; ++s) {
    if (s == R / 2 && t != 0) break;
    const int k = (s < R / 2) ? t + s * TL : N / 2;
    const cpx<T> zk = L[lds_idx(k)];
    const cpx<T> zm = conj(L[lds_idx((N - k) & (N - 1))]);
    const cpx<T> sum = zk + zm, dif = zk - zm;
    if (va) gstore(A + k, sum);
    if (vb) gstore(B + k, cpx<T>{dif.im, -dif.re});
  }
  __syncthreads();
}

// Row-pair passes reach half-spectrum rows ([rows][N/2+1] complex) through
// a buffer resource based at the block's first row; a thread passes the
// byte offset of its row, or kNoRow for a row past the end (loads read
// zeros, stores are dropped by the hardware range check).
constexpr unsigned kNoRow = 0x80000000u;

template <typename T, int N>
__device__ __forceinline__ FieldBuf pair_rows(const void* array, int first_row, int rows) {
  constexpr size_t rb = (size_t)(N / 2 + 1) * sizeof(cpx<T>);
  return FieldBuf((const char*)array + (size_t)first_row * rb, (unsigned)(rows * rb));
}
template <typename T, int N>
__device__ __forceinline__ unsigned pair_row_off(int row_in_block, bool valid) {
  return valid ? (unsigned)(row_in_block * (N / 2 + 1) * (int)sizeof(cpx<T>)) : kNoRow;
}
// Offset of row `row_in_block` in the pair-interleaved layout (see ColArr):
// the pair's base plus one element for the odd row; elements then step by
// two (kstep = 2 sizeof(cpx<T>) in the pair helpers below).
template <typename T, int N>
__device__ __forceinline__ unsigned pair_row_off_il(int row_in_block, bool valid) {
  return valid ? (unsigned)(((row_in_block & ~1) * (N / 2 + 1) + (row_in_block & 1)) * (int)sizeof(cpx<T>))
               : kNoRow;
}

// Gather z's spectrum from the half spectra A, B (n/2+1 entries each) of
// rows a and b: Z[k] = A[k] + i B[k], Z[n-k] = conj(A[k]) + i conj(B[k]).
// The imaginary parts of the self-conjugate modes k = 0, n/2 are ignored,
// as an inverse real transform does.  Row a starts at byte offset oa of
// buffer A, row b at ob of B, element k k * kstep bytes further; a missing
// row (offset kNoRow) reads as zero.
template <typename T, int N>
__device__ __forceinline__ void load_pair_spectrum_b(cpx<T> (&v)[line_radix(N)], const FieldBuf& A, unsigned oa,
                                                     const FieldBuf& B, unsigned ob, int t, T scale,
                                                     unsigned kstep = sizeof(cpx<T>)) {
  constexpr int TL = N / line_radix(N);
#pragma unroll
  for (int s = 0; s < line_radix(N); ++s) {
    const int e = t + s * TL;
    const bool lo = e <= N / 2;
    const unsigned k = (unsigned)(lo ? e : N - e) * kstep;
    cpx<T> a = A.template ldc<T>(oa + k, 0);
    cpx<T> b = B.template ldc<T>(ob + k, 0);
    if (e == 0 || e == N / 2) {
      a.im = 0;
      b.im = 0;
    }
    if (!lo) {
      a = conj(a);
      b = conj(b);
    }
    v[s] = (a + mul_i(b)) * scale;
  }
}

// load_pair_spectrum_b for a pair stored interleaved (element k of rows a
// and b side by side at byte offset o + 2k sizeof(cpx<T>); both rows present,
// or o = kNoRow for neither): one access per element pair.
template <typename T, int N>
__device__ __forceinline__ void load_pair_spectrum_il(cpx<T> (&v)[line_radix(N)], const FieldBuf& A, unsigned o,
                                                      int t, T scale) {
  constexpr int TL = N / line_radix(N);
  constexpr unsigned kstep = 2 * sizeof(cpx<T>);
#pragma unroll
  for (int s = 0; s < line_radix(N); ++s) {
    const int e = t + s * TL;
    const bool lo = e <= N / 2;
    cpx<T> a, b;
    A.ld2(o + (unsigned)(lo ? e : N - e) * kstep, a, b);
    if (e == 0 || e == N / 2) {
      a.im = 0;
      b.im = 0;
    }
    if (!lo) {
      a = conj(a);
      b = conj(b);
    }
    v[s] = (a + mul_i(b)) * scale;
  }
}

// store_pair_halves through buffers (rows at byte offsets oa, ob; element k
// k * kstep bytes further; a row at kNoRow is not stored).
template <typename T, int N>
__device__ __forceinline__ void store_pair_halves_b(const cpx<T> (&v)[line_radix(N)], cpx<T>* L, int t,
                                                    const FieldBuf& A, unsigned oa, const FieldBuf& B, unsigned ob,
                                                    unsigned kstep = sizeof(cpx<T>)) {
  constexpr int R = line_radix(N);
  constexpr int TL = N / R;
  __syncthreads();
#pragma unroll
  for (int s = 0; s < R; ++s) L[lds_idx(t + s * TL)] = v[s];
  __syncthreads();
#pragma unroll
  for (int s = 0; s <= R / 2; ++s) {
    if (s == R / 2 && t != 0) break;
    const int k = (s < R / 2) ? t + s * TL : N / 2;
    const cpx<T> zk = L[lds_idx(k)];
    const cpx<T> zm = conj(L[lds_idx((N - k) & (N - 1))]);
    const cpx<T> sum = zk + zm, dif = zk - zm;
    const unsigned kb = (unsigned)k * kstep;
    A.st(oa + kb, 0, sum);
    B.st(ob + kb, 0, cpx<T>{dif.im, -dif.re});
  }
  __syncthreads();
}

// store_pair_halves_b for a pair stored interleaved (see
// load_pair_spectrum_il): one access per element pair.
template <typename T, int N>
__device__ __forceinline__ void store_pair_halves_il(const cpx<T> (&v)[line_radix(N)], cpx<T>* L, int t,
                                                     const FieldBuf& A, unsigned o) {
  constexpr int R = line_radix(N);
  constexpr int TL = N / R;
  constexpr unsigned kstep = 2 * sizeof(cpx<T>);
  __syncthreads();
#pragma unroll
  for (int s = 0; s < R; ++s) L[lds_idx(t + s * TL)] = v[s];
  __syncthreads();
#pragma unroll
  for (int s = 0; s <= R / 2; ++s) {
    if (s == R / 2 && t != 0) break;
    const int k = (s < R / 2) ? t + s * TL : N / 2;
    const cpx<T> zk = L[lds_idx(k)];
    const cpx<T> zm = conj(L[lds_idx((N - k) & (N - 1))]);
    const cpx<T> sum = zk + zm, dif = zk - zm;
    A.st2(o + (unsigned)k * kstep, sum, cpx<T>{dif.im, -dif.re});
  }
  __syncthreads();
}

// ---------------------------------------------------------- N dispatch ---
template <int N>
using IntC = std::integral_constant<int, N>;

template <class F>
bool dispatch_n(int n, F&& f) {
  switch (n) {
    case 4: f(IntC<4>{}); return true;
    case 8: f(IntC<8>{}); return true;
    case 16: f(IntC<16>{}); return true;
    case 32: f(IntC<32>{}); return true;
    case 64: f(IntC<64>{}); return true;
    case 128: f(IntC<128>{}); return true;
    case 256: f(IntC<256>{}); return true;
    case 512: f(IntC<512>{}); return true;
    case 1024: f(IntC<1024>{}); return true;
    case 2048: f(IntC<2048>{}); return true;
    case 4096: f(IntC<4096>{}); return true;
    case 8192: f(IntC<8192>{}); return true;
    default: return false;
  }
}

}  // namespace pst
