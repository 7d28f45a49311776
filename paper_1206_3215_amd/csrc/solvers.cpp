// Solver drivers of the C ABI: launch sequences of the fused passes.
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <complex>
#include <utility>
#include <vector>

#include "launch.hpp"
#include "runtime.hpp"

using namespace pst;

namespace {

// exp(-i k^2 tau) - 1 = (cos - 1, -sin) for the n wavenumbers of a period,
// in double (cos - 1 as -2 sin^2 for accuracy at small angles).
std::vector<std::complex<double>> propagator_m1(int n, double length, double tau) {
  std::vector<std::complex<double>> e(n);
  for (int m = 0; m < n; ++m) {
    const double k = wavenumber(m, n, length);
    const double ph = k * k * tau;
    const double sh = std::sin(0.5 * ph);
    e[m] = std::complex<double>(-2.0 * sh * sh, -std::sin(ph));
  }
  return e;
}

pst_status nls_tables(Plan* pl, const pst_nls_params* p) {
  NlsTables& t = pl->nls;
  if (t.valid && t.dt == p->dt && t.lx == p->d.lx && t.ly == p->d.ly) return PST_OK;
  pst_status st = upload_complex(pl, propagator_m1(pl->nx, p->d.lx, 0.5 * p->dt), &t.ex_half, false, 1.0);
  if (st == PST_OK) st = upload_complex(pl, propagator_m1(pl->nx, p->d.lx, p->dt), &t.ex_full, false, 1.0);
  if (st == PST_OK) st = upload_complex(pl, propagator_m1(pl->ny, p->d.ly, 0.5 * p->dt), &t.ey_half, false, 1.0);
  if (st == PST_OK) st = upload_complex(pl, propagator_m1(pl->ny, p->d.ly, p->dt), &t.ey_full, false, 1.0);
  if (st != PST_OK) return st;
  t.valid = true;
  t.dt = p->dt;
  t.lx = p->d.lx;
  t.ly = p->d.ly;
  return PST_OK;
}

pst_status need_kind(Plan* pl, pst_kind k, const char* who) {
  if (pl == nullptr) return fail(PST_ERR_INVALID, "%s: plan is NULL", who);
  if (pl->kind != k)
    return fail(PST_ERR_INVALID, "%s needs a %s plan", who, k == PST_C2C ? "C2C" : "R2C");
  return PST_OK;
}

#define TRY(expr)                       \
  do {                                  \
    pst_status st_ = (expr);            \
    if (st_ != PST_OK) return st_;      \
  } while (0)

}  // namespace

extern "C" {

pst_status nls_step(pst_plan pl, void* psi, const pst_nls_params* p, int nsteps) {
  TRY(need_kind(pl, PST_C2C, "nls_step"));
  TRY(check_field(psi, "psi"));
  if (p == nullptr) return fail(PST_ERR_INVALID, "params is NULL");
  TRY(check_domain(p->d));
  if (!(p->dt != 0.0) || !std::isfinite(p->dt)) return fail(PST_ERR_INVALID, "dt must be finite and nonzero");
  if (!std::isfinite(p->g)) return fail(PST_ERR_INVALID, "g must be finite");
  if (nsteps < 0) return fail(PST_ERR_INVALID, "nsteps must be >= 0");
  if (nsteps == 0) return PST_OK;
  TRY(nls_tables(pl, p));
  const int nx = pl->nx, ny = pl->ny, B = pl->batch, W = pl->Wcol;
  const int lines = B * ny;
  const double pc = p->g * p->dt / ((double)nx * nx);
  const NlsTables& t = pl->nls;
  hipStream_t s = pl->stream;
  auto row = [&](int mode, double pc_, double scale) {
    if (mode == 1) prof_begin(pl, PST_PASS_NLS_ROW);
    pst_status r = hip_check(nls_row(pl->P, nx, lines, psi, mode, pc_, scale, pl->tw_x, s), "nls row");
    if (mode == 1) prof_end(pl);
    return r;
  };
  auto col = [&](const void* ex, const void* ey) {
    prof_begin(pl, PST_PASS_NLS_COL);
    pst_status r = hip_check(nls_col(pl->P, ny, nx, B, psi, pl->tw_y, ex, ey, W, s), "nls column");
    prof_end(pl);
    return r;
  };
  TRY(row(0, 0.0, (double)nx));
  TRY(col(t.ex_half, t.ey_half));
  for (int i = 1; i < nsteps; ++i) {
    TRY(row(1, pc, 1.0));
    TRY(col(t.ex_full, t.ey_full));
  }
  TRY(row(1, pc, 1.0));
  TRY(col(t.ex_half, t.ey_half));
  return row(2, 0.0, 1.0 / nx);
}

pst_status conserved_quantities(pst_plan pl, pst_eq eq, const void* f0, const void* f1,
                                const void* params, double* out) {
  if (pl == nullptr || params == nullptr || out == nullptr)
    return fail(PST_ERR_INVALID, "NULL argument");
  TRY(check_field(f0, "f0"));
  TRY(ensure_workspace(pl));
  const int nx = pl->nx, ny = pl->ny, B = pl->batch;
  hipStream_t s = pl->stream;
  double* rowp = static_cast<double*>(ws_at(pl, pl->off_rowpart));
  double* colp = static_cast<double*>(ws_at(pl, pl->off_colpart));
  if (eq == PST_NLS) {
    TRY(need_kind(pl, PST_C2C, "conserved_quantities(NLS)"));
    const pst_nls_params* p = static_cast<const pst_nls_params*>(params);
    TRY(check_domain(p->d));
    void* spec = ws_at(pl, pl->off_spec);
    const double dxdy = (p->d.lx / nx) * (p->d.ly / ny);
    const double kin = 0.5 * p->d.lx * p->d.ly / ((double)nx * ny * (double)nx * ny);
    TRY(hip_check(nls_cq_row(pl->P, nx, B * ny, f0, spec, rowp, pl->tw_x, s), "cq row"));
    TRY(hip_check(nls_cq_col(pl->P, ny, nx, B, spec, colp, pl->tw_y, 2 * M_PI / p->d.lx,
                             2 * M_PI / p->d.ly, pl->Wcol, s),
                  "cq column"));
    TRY(hip_check(nls_cq_finish(B, ny, nx, rowp, colp, dxdy, kin, p->g, pl->dres, pl->dstatus, s), "cq finish"));
  } else if (eq == PST_SG) {
    TRY(need_kind(pl, PST_R2C, "conserved_quantities(SG)"));
    TRY(check_field(f1, "f1"));
    const pst_sg_params* p = static_cast<const pst_sg_params*>(params);
    TRY(check_domain(p->d));
    if (!(p->dt > 0.0)) return fail(PST_ERR_INVALID, "dt must be > 0");
    const int h = nx / 2 + 1;
    void* UB = ws_at(pl, pl->off_spec);
    const double dxdy = (p->d.lx / nx) * (p->d.ly / ny);
    // 1/2 (lx ly/(nx ny)^2) sum |k|^2 |ubar_hat|^2, the stored transform being 2 ubar_hat
    const double grad = 0.125 * p->d.lx * p->d.ly / ((double)nx * ny * (double)nx * ny);
    TRY(hip_check(sg_h_row(pl->P, nx, B * ny, f0, f1, UB, rowp, 1.0 / p->dt, pl->tw_x, s), "H row"));
    TRY(hip_check(sg_h_col(pl->P, ny, nx, B, UB, colp, pl->tw_y, 2 * M_PI / p->d.lx, 2 * M_PI / p->d.ly,
                           col_w(pl, ny), s),
                  "H column"));
    TRY(hip_check(sg_h_finish(B, ny / 2, h, rowp, colp, dxdy, grad, pl->dres, pl->dstatus, s), "H finish"));
  } else if (eq == PST_NS) {
    TRY(need_kind(pl, PST_R2C, "conserved_quantities(NS)"));
    const pst_ns_params* p = static_cast<const pst_ns_params*>(params);
    TRY(check_domain(p->d));
    const int h = nx / 2 + 1;
    void* XH = ws_at(pl, pl->off_spec4);
    const double n2 = (double)nx * ny;
    const double en = 0.5 * p->d.lx * p->d.ly / (n2 * n2);
    const double zz = 0.5 * (p->d.lx / nx) * (p->d.ly / ny) / n2;
    TRY(hip_check(fft_row_r2c(pl->P, nx, B * ny, f0, XH, pl->tw_x, s), "NS cq row"));
    TRY(hip_check(ns_cq_col(pl->P, ny, nx, B, XH, colp, 2 * M_PI / p->d.lx, 2 * M_PI / p->d.ly, pl->tw_y, col_w(pl, ny), s),
                  "NS cq column"));
    TRY(hip_check(ns_cq_finish(B, h, colp, en, zz, pl->dres, pl->dstatus, s), "NS cq finish"));
  } else {
    return fail(PST_ERR_INVALID, "unknown equation %d", (int)eq);
  }
  TRY(hip_check(hipMemcpyAsync(out, pl->dres, (size_t)B * 4 * sizeof(double), hipMemcpyDeviceToHost, s),
                "read results"));
  TRY(hip_check(hipStreamSynchronize(s), "hipStreamSynchronize"));
  for (int i = 0; i < 4 * B; ++i)
    if (!std::isfinite(out[i])) return fail(PST_ERR_NONFINITE, "conserved quantity is not finite");
  return PST_OK;
}

static pst_status sg_check(Plan* pl, const pst_sg_params* p, const char* who) {
  TRY(need_kind(pl, PST_R2C, who));
  if (p == nullptr) return fail(PST_ERR_INVALID, "%s: params is NULL", who);
  TRY(check_domain(p->d));
  if (!(p->dt > 0.0) || !std::isfinite(p->dt)) return fail(PST_ERR_INVALID, "%s: dt must be finite and > 0", who);
  return ensure_workspace(pl);
}

pst_status sg_start(pst_plan pl, const void* u0, const void* v0, void* u_prev, void* u_curr,
                    const pst_sg_params* p) {
  TRY(sg_check(pl, p, "sg_start"));
  TRY(check_field(u0, "u0"));
  TRY(check_field(v0, "v0"));
  TRY(check_field(u_prev, "u_prev"));
  TRY(check_field(u_curr, "u_curr"));
  if (u_prev == u_curr) return fail(PST_ERR_INVALID, "sg_start: u_prev and u_curr must differ");
  if (u_curr == u0 || u_prev == v0) return fail(PST_ERR_INVALID, "sg_start: outputs alias the wrong inputs");
  const int nx = pl->nx, ny = pl->ny, B = pl->batch, lines = B * ny;
  void* U = ws_at(pl, pl->off_spec);
  void* S = ws_at(pl, pl->off_spec2);
  void* W = ws_at(pl, pl->off_spec3);
  const double sc = 0.5 / ((double)nx * ny), dt = p->dt;
  hipStream_t s = pl->stream;
  TRY(hip_check(sg_row(pl->P, 0, nx, lines, nullptr, u0, nullptr, 0.0, nullptr, nullptr, nullptr, U, S, pl->tw_x, s),
                "sg entry row"));
  // u^1 - u^0 = iFFT((c1s - 1) U - c2s S) + dt v0, c1s = (1-a)/(1+a), c2s = dt^2/(2(1+a))
  TRY(hip_check(sg_col(pl->P, ny, nx, B, U, S, W, pl->tw_y, 2 * M_PI / p->d.lx, 2 * M_PI / p->d.ly,
                       0.25 * dt * dt, 1.0, 0.5 * dt * dt, sc, col_w(pl, ny), s),
                "sg start column"));
  return hip_check(sg_row(pl->P, 2, nx, lines, W, u0, v0, dt, u_curr, nullptr, u_prev, nullptr, nullptr, pl->tw_x, s),
                   "sg start row");
}

pst_status sg_step(pst_plan pl, void* u_prev, void* u_curr, const pst_sg_params* p, int nsteps) {
  TRY(sg_check(pl, p, "sg_step"));
  TRY(check_field(u_prev, "u_prev"));
  TRY(check_field(u_curr, "u_curr"));
  if (u_prev == u_curr) return fail(PST_ERR_INVALID, "sg_step: u_prev and u_curr must differ");
  if (nsteps < 0) return fail(PST_ERR_INVALID, "nsteps must be >= 0");
  if (nsteps == 0) return PST_OK;
  const int nx = pl->nx, ny = pl->ny, B = pl->batch, lines = B * ny;
  void* U = ws_at(pl, pl->off_spec);
  void* S = ws_at(pl, pl->off_spec2);
  void* W = ws_at(pl, pl->off_spec3);
  const double sc = 0.5 / ((double)nx * ny), dt = p->dt;
  const double kx0 = 2 * M_PI / p->d.lx, ky0 = 2 * M_PI / p->d.ly;
  const int Wt = col_w(pl, ny);
  hipStream_t s = pl->stream;
  auto col = [&]() {
    prof_begin(pl, PST_PASS_SG_COL);
    pst_status r = hip_check(sg_col(pl->P, ny, nx, B, U, S, W, pl->tw_y, kx0, ky0, 0.25 * dt * dt, 2.0, dt * dt, sc,
                                    Wt, s),
                             "sg column");
    prof_end(pl);
    return r;
  };
  // u_curr holds u^n; u_prev's buffer holds the increment d^n during the call
  TRY(hip_check(sg_row(pl->P, 0, nx, lines, nullptr, u_curr, u_prev, 0.0, nullptr, u_prev, nullptr, U, S, pl->tw_x, s),
                "sg entry row"));
  TRY(col());
  for (int i = 0; i < nsteps - 1; ++i) {
    prof_begin(pl, PST_PASS_SG_ROW);
    TRY(hip_check(sg_row(pl->P, 1, nx, lines, W, u_curr, u_prev, 1.0, u_curr, u_prev, nullptr, U, S, pl->tw_x, s),
                  "sg row"));
    prof_end(pl);
    TRY(col());
  }
  // last step: u_curr <- u^N, u_prev <- u^{N-1} (the level it replaces)
  return hip_check(sg_row(pl->P, 2, nx, lines, W, u_curr, u_prev, 1.0, u_curr, nullptr, u_prev, nullptr, nullptr,
                          pl->tw_x, s),
                   "sg final row");
}

pst_status ns_step(pst_plan pl, void* omega, const pst_ns_params* p, int nsteps, int* dev_iters) {
  TRY(need_kind(pl, PST_R2C, "ns_step"));
  TRY(check_field(omega, "omega"));
  if (p == nullptr) return fail(PST_ERR_INVALID, "params is NULL");
  TRY(check_domain(p->d));
  if (!(p->dt > 0.0) || !std::isfinite(p->dt)) return fail(PST_ERR_INVALID, "dt must be finite and > 0");
  if (!(p->nu >= 0.0) || !std::isfinite(p->nu)) return fail(PST_ERR_INVALID, "nu must be finite and >= 0");
  if (!(p->tol >= 0.0)) return fail(PST_ERR_INVALID, "tol must be >= 0");
  if (p->max_iter < 1 || p->max_iter > 10000) return fail(PST_ERR_INVALID, "max_iter must be in [1, 10000]");
  if (p->fixed_iters < 0 || p->fixed_iters > 10000) return fail(PST_ERR_INVALID, "fixed_iters must be in [0, 10000]");
  if (nsteps < 0) return fail(PST_ERR_INVALID, "nsteps must be >= 0");
  if (nsteps == 0) return PST_OK;
  TRY(ensure_workspace(pl));
  const int nx = pl->nx, ny = pl->ny, B = pl->batch, lines = B * ny, h = nx / 2 + 1;
  const int Wt = col_w(pl, ny);
  hipStream_t s = pl->stream;
  NsPtrs P;
  P.Q = ws_at(pl, pl->off_spec);
  P.WN = ws_at(pl, pl->off_spec2);
  P.DK = ws_at(pl, pl->off_spec3);
  P.NH = ws_at(pl, pl->off_spec4);
  P.OUT = ws_at(pl, pl->off_spec4);
  P.D = ws_at(pl, pl->off_hyb);
  P.dstride = (size_t)B * ny * h;
  P.part = static_cast<double*>(ws_at(pl, pl->off_colpart));
  NsScalars S;
  S.kx0 = 2 * M_PI / p->d.lx;
  S.ky0 = 2 * M_PI / p->d.ly;
  S.hnu = 0.5 * p->dt * p->nu;
  S.qdt = 0.5 * p->dt;
  S.nscale = 0.5;
  S.dscale = 1.0 / ((double)nx * ny);
  S.nx = nx;
  S.kx_cut = (nx - 1) / 3;
  S.ky_cut = (ny - 1) / 3;
  int* done = static_cast<int*>(ws_at(pl, pl->off_nsstate));
  int* iters = done + B;
  double* resid = reinterpret_cast<double*>(static_cast<char*>(ws_at(pl, pl->off_nsstate)) +
                                            ((2 * B * sizeof(int) + 7) & ~(size_t)7));
  const double vol = (p->d.lx / nx) * (p->d.ly / ny) / ((double)nx * ny);
  const double eps = pl->prec == PST_FP32 ? std::ldexp(1.0, -23) : 0.0;
  const double fp_floor = (16 * eps) * (16 * eps);
  const int fixed = p->fixed_iters;
  auto row = [&](const int* gate) {
    prof_begin(pl, PST_PASS_NS_ROW);
    pst_status r = hip_check(ns_row(pl->P, nx, lines, ny, P.D, P.dstride, (void*)P.NH, gate, pl->tw_x, s), "ns row");
    prof_end(pl);
    return r;
  };
  auto col = [&](int mode) {
    if (mode == 1 || mode == 2) prof_begin(pl, PST_PASS_NS_COL);
    pst_status r = hip_check(ns_col(pl->P, mode, ny, B, P, S, done, pl->tw_y, Wt, s), "ns column");
    if (mode == 1 || mode == 2) prof_end(pl);
    return r;
  };
  auto finish = [&](int first, int* iters_out) {
    return hip_check(ns_finish(B, h, P.part, vol, p->tol, fp_floor, p->max_iter, fixed, first, done, iters,
                               iters_out, resid, pl->dstatus, s),
                     "ns finish");
  };
  // entry: w^n = rfft2(omega), increment 0, derivatives of w^n
  TRY(hip_check(fft_row_r2c(pl->P, nx, lines, omega, (void*)P.NH, pl->tw_x, s), "ns entry row"));
  TRY(col(0));
  std::vector<int> hbuf(2 * B);
  for (int step = 0; step < nsteps; ++step) {
    int* iout = dev_iters ? dev_iters + (size_t)step * B : nullptr;
    TRY(row(nullptr));
    TRY(col(1));
    TRY(finish(1, iout));
    int launched = 1;
    const int target = fixed > 0 ? fixed : std::min(std::max(pl->ns_guess, 1), p->max_iter);
    while (launched < target) {
      TRY(row(done));
      TRY(col(2));
      TRY(finish(0, iout));
      ++launched;
    }
    if (fixed > 0) continue;
    int most = 0;
    while (true) {
      TRY(hip_check(hipMemcpyAsync(hbuf.data(), done, 2 * B * sizeof(int), hipMemcpyDeviceToHost, s), "read ns flags"));
      TRY(hip_check(hipStreamSynchronize(s), "hipStreamSynchronize"));
      bool all = true;
      most = 0;
      for (int f = 0; f < B; ++f) {
        all = all && hbuf[f] != 0;
        most = std::max(most, hbuf[B + f]);
      }
      if (all || launched >= p->max_iter) break;
      TRY(row(done));
      TRY(col(2));
      TRY(finish(0, iout));
      ++launched;
    }
    pl->ns_guess = std::max(1, most);
  }
  // exit: omega = irfft2(w^n + d)
  TRY(col(3));
  return hip_check(fft_row_c2r(pl->P, nx, lines, P.OUT, omega, 1.0 / ((double)nx * ny), pl->tw_x, s), "ns exit row");
}

pst_status solve_batch(const pst_request*, int, void*) {
  return fail(PST_ERR_UNSUPPORTED, "solve_batch: not available yet");
}

}  // extern "C"
