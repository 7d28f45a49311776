// Host runtime of the pst library: plans, tables, validation and the C ABI
// declared in include/pst.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "fft_line.hpp"
#include "launch.hpp"
#include "pst.h"
#include "runtime.hpp"

namespace pst {

thread_local std::string g_last_error;

pst_status fail(pst_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

pst_status hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return PST_OK;
  if (e == hipErrorOutOfMemory) return fail(PST_ERR_OOM, "%s: %s", what, hipGetErrorString(e));
  return fail(PST_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

int size_class(int n) {
  if (n < 4 || n > 8192) return 0;
  if ((n & (n - 1)) == 0) return 1;
  int m = n;
  for (int f : {2, 3, 5})
    while (m % f == 0) m /= f;
  return m == 1 ? 2 : 0;
}

// Stage list of a mixed-radix line (layout in launch.hpp): radix-5 and
// radix-3 stages first, then radix 8 while it divides, then a 4 or a 2.
static MixedLine mixed_line(int n) {
  MixedLine ml;
  ml.n = n;
  int m = n, ns = 1, off = 0;
  auto push = [&](int r) {
    ml.r[ml.nst] = r;
    ml.ns[ml.nst] = ns;
    ml.toff[ml.nst] = off;
    if (ml.nst > 0) off += (r - 1) * ns;
    ns *= r;
    ++ml.nst;
    m /= r;
  };
  while (m % 5 == 0) push(5);
  while (m % 3 == 0) push(3);
  while (m % 8 == 0) push(8);
  if (m % 4 == 0) push(4);
  if (m % 2 == 0) push(2);
  return ml;
}

// Twiddle table of a mixed-radix line, in double precision.
static std::vector<std::complex<double>> mixed_twiddles(const MixedLine& ml) {
  size_t len = 1;
  for (int s = 1; s < ml.nst; ++s) len = std::max(len, (size_t)ml.toff[s] + (size_t)(ml.r[s] - 1) * ml.ns[s]);
  std::vector<std::complex<double>> tab(len);
  for (int s = 1; s < ml.nst; ++s) {
    const int r = ml.r[s], ns = ml.ns[s];
    const long M = (long)ns * r;
    for (int q = 1; q < r; ++q)
      for (int k = 0; k < ns; ++k) {
        const long mm = ((long)q * k) % M;
        const double ang = -2.0 * M_PI * (double)mm / (double)M;
        tab[ml.toff[s] + (q - 1) * ns + k] = {std::cos(ang), std::sin(ang)};
      }
  }
  return tab;
}

// Twiddle table of the line FFT of length n (layout in fft_line.hpp: the
// stages of the default radix, then those of radix 8 where compiled), in
// double precision, rounded once to the plan's precision.
static std::vector<std::complex<double>> twiddles(int n) {
  std::vector<std::complex<double>> tab(tw_table_total(n) > 0 ? tw_table_total(n) : 1);
  auto fill = [&](int R) {
    const int base = tw_base(n, R);
    for (int s = 1; s < num_stages(n, R); ++s) {
      const int r = stage_radix(n, R, s), ns = stage_ns(n, R, s), off = base + stage_tw_offset(n, R, s);
      const long M = (long)ns * r;
      for (int q = 1; q < r; ++q)
        for (int k = 0; k < ns; ++k) {
          const long m = ((long)q * k) % M;
          const double ang = -2.0 * M_PI * (double)m / (double)M;
          tab[off + (q - 1) * ns + k] = {std::cos(ang), std::sin(ang)};
        }
    }
  };
  fill(line_radix(n));
  if (has_radix8(n)) fill(8);
  return tab;
}

// Round a unit-modulus complex number to single precision: among the float
// pairs within two ulps of (cos, sin) whose angle is within 6e-8 rad of the
// exact one, take the pair whose modulus is closest to 1 (nearest rounding
// gives |w|^2 - 1 up to ~6e-8).  FFT round trips then carry no systematic
// gain, which would otherwise act at every time step.
static void round_unit(std::complex<double> z, float* re, float* im) {
  const double a = z.real(), b = z.imag(), ang0 = std::atan2(b, a);
  float ac[5], bc[5];
  ac[0] = (float)a;
  bc[0] = (float)b;
  for (int i = 1; i <= 2; ++i) {
    ac[2 * i - 1] = std::nextafter(ac[2 * i - 3 < 0 ? 0 : 2 * i - 3], -2.0f);
    ac[2 * i] = std::nextafter(ac[2 * i - 2], 2.0f);
    bc[2 * i - 1] = std::nextafter(bc[2 * i - 3 < 0 ? 0 : 2 * i - 3], -2.0f);
    bc[2 * i] = std::nextafter(bc[2 * i - 2], 2.0f);
  }
  double best = 1e300;
  *re = ac[0];
  *im = bc[0];
  for (float x : ac)
    for (float y : bc) {
      double da = std::atan2((double)y, (double)x) - ang0;
      da = std::remainder(da, 2.0 * M_PI);
      if (std::fabs(da) > 6e-8) continue;
      const double e = std::fabs((double)x * x + (double)y * y - 1.0);
      if (e < best) {
        best = e;
        *re = x;
        *im = y;
      }
    }
}

// Upload complex doubles as the plan's precision.  unit: entries are
// exp(i phi) * scale with scale a power of two (see round_unit).
pst_status upload_complex(Plan* pl, const std::vector<std::complex<double>>& h, void** dptr, bool unit,
                          double scale) {
  const size_t n = h.size();
  std::vector<char> buf(n * pl->csize);
  if (pl->prec == PST_FP32) {
    float* f = reinterpret_cast<float*>(buf.data());
    for (size_t i = 0; i < n; ++i) {
      if (unit) {
        round_unit(h[i], &f[2 * i], &f[2 * i + 1]);
        f[2 * i] *= (float)scale;
        f[2 * i + 1] *= (float)scale;
      } else {
        f[2 * i] = (float)(h[i].real() * scale);
        f[2 * i + 1] = (float)(h[i].imag() * scale);
      }
    }
  } else {
    double* d = reinterpret_cast<double*>(buf.data());
    for (size_t i = 0; i < n; ++i) {
      d[2 * i] = h[i].real() * scale;
      d[2 * i + 1] = h[i].imag() * scale;
    }
  }
  if (*dptr == nullptr) {
    pst_status st = hip_check(hipMalloc(dptr, buf.size()), "hipMalloc(table)");
    if (st != PST_OK) return st;
    pl->owned.push_back(*dptr);
  }
  return hip_check(hipMemcpy(*dptr, buf.data(), buf.size(), hipMemcpyHostToDevice), "upload table");
}

double wavenumber(int m, int n, double length) {
  // m in {0..n/2-1, -n/2..-1} for even n, {0..(n-1)/2, -(n-1)/2..-1} for odd n
  const int mm = m < (n + 1) / 2 ? m : m - n;
  return 2.0 * M_PI * (double)mm / length;
}

pst_status check_domain(const pst_domain& d) {
  if (!(d.lx > 0.0) || !(d.ly > 0.0) || !std::isfinite(d.lx) || !std::isfinite(d.ly) ||
      !std::isfinite(d.x0) || !std::isfinite(d.y0))
    return fail(PST_ERR_INVALID, "domain periods must be finite and > 0");
  return PST_OK;
}

pst_status check_field(const void* p, const char* name) {
  if (p == nullptr) return fail(PST_ERR_INVALID, "%s is NULL", name);
  if (reinterpret_cast<uintptr_t>(p) % 256 != 0) return fail(PST_ERR_INVALID, "%s is not 256-byte aligned", name);
  return PST_OK;
}

pst_status ensure_workspace(Plan* pl) {
  if (pl->ws != nullptr) return PST_OK;
  pst_status st = hip_check(hipMalloc(&pl->ws, pl->ws_need), "hipMalloc(workspace)");
  if (st != PST_OK) return st;
  pl->ws_owned = true;
  return PST_OK;
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Workspace: a list of regions, each 256-byte aligned.
size_t ws_layout(Plan* pl) {
  const size_t B = pl->batch, nx = pl->nx, ny = pl->ny, h = nx / 2 + 1;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align256(bytes);
    return o;
  };
  if (pl->kind == PST_C2C) {
    pl->off_spec = take(B * ny * nx * pl->csize);
    pl->off_rowpart = take(B * ny * 2 * sizeof(double));
    pl->off_colpart = take(B * nx * sizeof(double));
  } else {
    // Fields of the real solvers; see the sine-Gordon and Navier-Stokes drivers.
    pl->off_spec = take(B * ny * h * pl->csize);
    pl->off_spec2 = take(B * ny * h * pl->csize);
    pl->off_spec3 = take(B * ny * h * pl->csize);
    pl->off_spec4 = take(B * ny * h * pl->csize);
    pl->off_hyb = take(4 * B * ny * h * pl->csize);
    pl->off_rowpart = take(B * ny * 4 * sizeof(double));
    pl->off_colpart = take(B * h * 4 * sizeof(double));
    // Navier-Stokes per-field state: done, iters, park, park_step, maxit, resid
    pl->off_nsstate = take(B * (5 * sizeof(int) + sizeof(double)) + 64);
  }
  return off;
}

static hipEvent_t take_event(Plan* pl) {
  if (pl->ev_used == pl->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    pl->ev_pool.push_back(e);
  }
  return pl->ev_pool[pl->ev_used++];
}

static int g_prof_pass = -1;
static hipEvent_t g_prof_start = nullptr;

void prof_begin(Plan* pl, int pass) {
  if (!pl->prof) return;
  g_prof_start = take_event(pl);
  g_prof_pass = pass;
  // Profiling is best effort: a pass whose start cannot be recorded is not timed.
  if (g_prof_start && hipEventRecord(g_prof_start, pl->stream) != hipSuccess) g_prof_start = nullptr;
}

void prof_end(Plan* pl) {
  if (!pl->prof || g_prof_start == nullptr) return;
  hipEvent_t e = take_event(pl);
  if (e == nullptr || hipEventRecord(e, pl->stream) != hipSuccess) {
    g_prof_start = nullptr;
    return;
  }
  pl->ev_rec.push_back({g_prof_pass, {g_prof_start, e}});
  g_prof_start = nullptr;
}

}  // namespace pst

using namespace pst;

extern "C" {

const char* pst_last_error(void) { return g_last_error.c_str(); }
const char* pst_version(void) { return "pst 0.1 (gfx950)"; }

pst_status fft2d_plan(int nx, int ny, pst_kind kind, pst_prec prec, int batch, void* hip_stream,
                      pst_plan* out) {
  if (out == nullptr) return fail(PST_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!size_class(nx) || !size_class(ny))
    return fail(PST_ERR_INVALID, "nx=%d, ny=%d: sizes must be 2^a 3^b 5^c in [4, 8192]", nx, ny);
  if (kind != PST_C2C && kind != PST_R2C) return fail(PST_ERR_INVALID, "unknown kind %d", (int)kind);
  if (prec != PST_FP32 && prec != PST_FP64) return fail(PST_ERR_INVALID, "unknown precision %d", (int)prec);
  const bool mixed = size_class(nx) == 2 || size_class(ny) == 2;
  if (mixed && (!mixed_supported(prec == PST_FP32 ? P32 : P64, nx) || !mixed_supported(prec == PST_FP32 ? P32 : P64, ny)))
    return fail(PST_ERR_UNSUPPORTED, "nx=%d, ny=%d: lengths that are not powers of two are limited to %d (%s)", nx,
                ny, prec == PST_FP32 ? 9600 : 4800, prec == PST_FP32 ? "FP32" : "FP64");
  if (batch < 1 || batch > (1 << 20)) return fail(PST_ERR_INVALID, "batch=%d out of range", batch);
  Plan* pl = new Plan();
  pl->nx = nx;
  pl->ny = ny;
  pl->kind = kind;
  pl->prec = prec;
  pl->batch = batch;
  pl->stream = reinterpret_cast<hipStream_t>(hip_stream);
  pl->csize = prec == PST_FP32 ? 8 : 16;
  pl->rsize = prec == PST_FP32 ? 4 : 8;
  pl->P = prec == PST_FP32 ? P32 : P64;
  pl->mixed = mixed;
  pst_status st = hip_check(hipGetDevice(&pl->device), "hipGetDevice");
  if (mixed) {
    // every pass of a plan with a non-power-of-two length runs the
    // mixed-radix kernels, for both axes
    pl->mlx = mixed_line(nx);
    pl->mly = mixed_line(ny);
    if (st == PST_OK) st = upload_complex(pl, mixed_twiddles(pl->mlx), &pl->tw_x, true, 1.0);
    if (st == PST_OK) st = upload_complex(pl, mixed_twiddles(pl->mly), &pl->tw_y, true, 1.0);
  } else {
    if (st == PST_OK) st = upload_complex(pl, twiddles(nx), &pl->tw_x, true, 1.0);
    if (st == PST_OK) st = upload_complex(pl, twiddles(ny), &pl->tw_y, true, 1.0);
  }
  if (st == PST_OK) {
    void* p = nullptr;
    st = hip_check(hipMalloc(&p, 256 + (size_t)batch * 8 * sizeof(double)), "hipMalloc(status)");
    if (st == PST_OK) {
      pl->owned.push_back(p);
      pl->dstatus = reinterpret_cast<int*>(p);
      pl->dres = reinterpret_cast<double*>(reinterpret_cast<char*>(p) + 256);
      st = hip_check(hipMemset(p, 0, 256), "hipMemset(status)");
    }
  }
  if (st != PST_OK) {
    fft2d_destroy(pl);
    return st;
  }
  pl->ws_need = ws_layout(pl);
  *out = pl;
  return PST_OK;
}

pst_status pst_workspace_size(pst_plan plan, size_t* bytes) {
  if (plan == nullptr || bytes == nullptr) return fail(PST_ERR_INVALID, "NULL argument");
  *bytes = plan->ws_need;
  return PST_OK;
}

pst_status pst_set_workspace(pst_plan plan, void* dev_ptr, size_t bytes) {
  if (plan == nullptr || dev_ptr == nullptr) return fail(PST_ERR_INVALID, "NULL argument");
  if (bytes < plan->ws_need)
    return fail(PST_ERR_INVALID, "workspace of %zu bytes is smaller than the %zu needed", bytes, plan->ws_need);
  if (reinterpret_cast<uintptr_t>(dev_ptr) % 256 != 0) return fail(PST_ERR_INVALID, "workspace not 256-byte aligned");
  if (plan->ws_owned) {
    pst_status st = hip_check(hipStreamSynchronize(plan->stream), "hipStreamSynchronize");
    if (st != PST_OK) return st;  // the old workspace may still be in use: keep it
    (void)hipFree(plan->ws);
  }
  plan->ws = dev_ptr;
  plan->ws_owned = false;
  return PST_OK;
}

pst_status fft2d_destroy(pst_plan plan) {
  if (plan == nullptr) return fail(PST_ERR_INVALID, "plan is NULL");
  // The plan is released whatever happens; the first failure is reported.
  pst_status st = hip_check(hipStreamSynchronize(plan->stream), "hipStreamSynchronize");
  for (void* p : plan->owned) (void)hipFree(p);
  for (hipEvent_t e : plan->ev_pool) (void)hipEventDestroy(e);
  if (plan->ws_owned) (void)hipFree(plan->ws);
  if (plan->ns_host) (void)hipHostFree(plan->ns_host);
  if (plan->ns_ev) (void)hipEventDestroy(plan->ns_ev);
  delete plan;
  return st;
}

pst_status fft2d_exec(pst_plan pl, const void* in, void* out, int sign) {
  if (pl == nullptr) return fail(PST_ERR_INVALID, "plan is NULL");
  pst_status st = check_field(in, "in");
  if (st == PST_OK) st = check_field(out, "out");
  if (st != PST_OK) return st;
  if (sign != -1 && sign != 1) return fail(PST_ERR_INVALID, "sign must be -1 or +1");
  const int nx = pl->nx, ny = pl->ny, B = pl->batch, h = nx / 2 + 1;
  const bool inv = sign == 1;
  const double sc = inv ? 1.0 / ((double)nx * ny) : 1.0;
  if (pl->mixed) {
    if (pl->kind == PST_C2C) {
      st = hip_check(mixed_row_c2c(pl->P, pl->mlx, B * ny, in, out, inv, 1.0, pl->tw_x, pl->stream), "row pass");
      if (st != PST_OK) return st;
      return hip_check(mixed_col_c2c(pl->P, pl->mly, nx, nx, B, out, out, inv, sc, pl->tw_y, pl->stream),
                       "column pass");
    }
    if (in == out) return fail(PST_ERR_INVALID, "R2C transforms cannot run in place");
    if (!inv) {
      st = hip_check(mixed_row_r2c(pl->P, pl->mlx, B * ny, in, out, pl->tw_x, pl->stream), "r2c row pass");
      if (st != PST_OK) return st;
      return hip_check(mixed_col_c2c(pl->P, pl->mly, h, h, B, out, out, false, 1.0, pl->tw_y, pl->stream),
                       "column pass");
    }
    if ((st = ensure_workspace(pl)) != PST_OK) return st;
    void* tmp = ws_at(pl, pl->off_spec);
    st = hip_check(mixed_col_c2c(pl->P, pl->mly, h, h, B, in, tmp, true, 1.0, pl->tw_y, pl->stream), "column pass");
    if (st != PST_OK) return st;
    return hip_check(mixed_row_c2r(pl->P, pl->mlx, B * ny, tmp, out, sc, pl->tw_x, pl->stream), "c2r row pass");
  }
  if (pl->kind == PST_C2C) {
    st = hip_check(fft_row_c2c(pl->P, nx, B * ny, in, out, inv, 1.0, pl->tw_x, pl->stream), "row pass");
    if (st != PST_OK) return st;
    return hip_check(fft_col_c2c(pl->P, ny, nx, nx, B, out, out, inv, sc, pl->tw_y, pl->colvar, pl->stream),
                     "column pass");
  }
  if (in == out) return fail(PST_ERR_INVALID, "R2C transforms cannot run in place");
  if (!inv) {
    st = hip_check(fft_row_r2c(pl->P, nx, B * ny, ny, contiguous(in, (size_t)nx * ny * pl->rsize), out, pl->tw_x,
                               pl->stream),
                   "r2c row pass");
    if (st != PST_OK) return st;
    return hip_check(fft_col_c2c(pl->P, ny, h, h, B, out, out, false, 1.0, pl->tw_y, col_w(pl, ny), pl->stream),
                     "column pass");
  }
  if ((st = ensure_workspace(pl)) != PST_OK) return st;
  void* tmp = ws_at(pl, pl->off_spec);
  st = hip_check(fft_col_c2c(pl->P, ny, h, h, B, in, tmp, true, 1.0, pl->tw_y, col_w(pl, ny), pl->stream),
                 "column pass");
  if (st != PST_OK) return st;
  return hip_check(fft_row_c2r(pl->P, nx, B * ny, ny, tmp, contiguous(out, (size_t)nx * ny * pl->rsize), sc, pl->tw_x,
                               pl->stream),
                   "c2r row pass");
}

pst_status pst_set_column_variant(pst_plan pl, int variant) {
  if (pl == nullptr) return fail(PST_ERR_INVALID, "plan is NULL");
  if (pl->mixed) {
    if (variant != 0) return fail(PST_ERR_INVALID, "mixed-radix plans have only column variant 0");
    return PST_OK;
  }
  int w, v, sp, r;
  if (!col_variant_info(pl->P, pl->ny, variant, pl->kind == PST_C2C, &w, &v, &sp, &r))
    return fail(PST_ERR_INVALID, "column variant %d is not compiled for ny=%d", variant, pl->ny);
  pl->colvar = variant;
  return PST_OK;
}

pst_status pst_set_row_variant(pst_plan pl, int variant) {
  if (pl == nullptr) return fail(PST_ERR_INVALID, "plan is NULL");
  int p, v, sp, r;
  if (pl->kind != PST_C2C || pl->mixed) {
    if (variant != 0) return fail(PST_ERR_INVALID, "R2C and mixed-radix plans have only row variant 0");
  } else if (!nls_row_variant_info(pl->P, pl->nx, variant, &p, &v, &sp, &r)) {
    return fail(PST_ERR_INVALID, "row variant %d is not compiled for nx=%d", variant, pl->nx);
  }
  pl->rowvar = variant;
  return PST_OK;
}

pst_status pst_get_variants(pst_plan pl, int* row_variant, int* column_variant) {
  if (pl == nullptr || row_variant == nullptr || column_variant == nullptr)
    return fail(PST_ERR_INVALID, "NULL argument");
  *row_variant = pl->rowvar;
  *column_variant = pl->colvar;
  return PST_OK;
}

pst_status pst_column_variant_info(pst_prec prec, int n, int variant, int single_field, int* columns,
                                   int* values_per_thread, int* split, int* radix) {
  if (prec != PST_FP32 && prec != PST_FP64) return fail(PST_ERR_INVALID, "unknown precision %d", (int)prec);
  if (columns == nullptr || values_per_thread == nullptr || split == nullptr || radix == nullptr)
    return fail(PST_ERR_INVALID, "output pointer is NULL");
  if (!col_variant_info(prec == PST_FP32 ? P32 : P64, n, variant, single_field != 0, columns, values_per_thread,
                        split, radix))
    return fail(PST_ERR_INVALID, "no column variant %d for length %d", variant, n);
  return PST_OK;
}

pst_status pst_row_variant_info(pst_prec prec, int n, int variant, int* pairs_per_block, int* values_per_thread,
                                int* split, int* radix) {
  if (prec != PST_FP32 && prec != PST_FP64) return fail(PST_ERR_INVALID, "unknown precision %d", (int)prec);
  if (pairs_per_block == nullptr || values_per_thread == nullptr || split == nullptr || radix == nullptr)
    return fail(PST_ERR_INVALID, "output pointer is NULL");
  if (!nls_row_variant_info(prec == PST_FP32 ? P32 : P64, n, variant, pairs_per_block, values_per_thread, split,
                            radix))
    return fail(PST_ERR_INVALID, "no row variant %d for length %d", variant, n);
  return PST_OK;
}

pst_status pst_profile_enable(pst_plan pl, int enable) {
  if (pl == nullptr) return fail(PST_ERR_INVALID, "plan is NULL");
  pl->prof = enable != 0;
  pl->ev_rec.clear();
  pl->ev_used = 0;
  return PST_OK;
}

pst_status pst_profile_read(pst_plan pl, int pass, double* total_ms, int* count) {
  if (pl == nullptr || total_ms == nullptr || count == nullptr) return fail(PST_ERR_INVALID, "NULL argument");
  if (pass < 0 || pass >= PST_PASS_COUNT) return fail(PST_ERR_INVALID, "unknown pass %d", pass);
  pst_status st = hip_check(hipStreamSynchronize(pl->stream), "hipStreamSynchronize");
  if (st != PST_OK) return st;
  double tot = 0.0;
  int n = 0;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> keep;
  for (auto& r : pl->ev_rec) {
    if (r.first != pass) {
      keep.push_back(r);
      continue;
    }
    float ms = 0.0f;
    st = hip_check(hipEventElapsedTime(&ms, r.second.first, r.second.second), "hipEventElapsedTime");
    if (st != PST_OK) return st;
    tot += ms;
    ++n;
  }
  pl->ev_rec.swap(keep);
  if (pl->ev_rec.empty()) pl->ev_used = 0;
  *total_ms = tot;
  *count = n;
  return PST_OK;
}

pst_status pst_sync_status(pst_plan pl, pst_status* device_status) {
  if (pl == nullptr || device_status == nullptr) return fail(PST_ERR_INVALID, "NULL argument");
  int h = 0;
  pst_status st = hip_check(hipMemcpyAsync(&h, pl->dstatus, sizeof(int), hipMemcpyDeviceToHost, pl->stream),
                            "read status");
  if (st == PST_OK) st = hip_check(hipStreamSynchronize(pl->stream), "hipStreamSynchronize");
  if (st == PST_OK) st = hip_check(hipMemsetAsync(pl->dstatus, 0, sizeof(int), pl->stream), "clear status");
  if (st != PST_OK) return st;
  *device_status = (h & ST_NONFINITE) ? PST_ERR_NONFINITE : (h & ST_NOT_CONVERGED) ? PST_ERR_NOT_CONVERGED : PST_OK;
  return PST_OK;
}

}  // extern "C"
