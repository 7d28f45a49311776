// Solver drivers of the C ABI: launch sequences of the fused passes.
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <complex>
#include <cstring>
#include <map>
#include <mutex>
#include <memory>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "launch.hpp"
#include "runtime.hpp"

using namespace pst;

#define TRY(expr)                       \
  do {                                  \
    pst_status st_ = (expr);            \
    if (st_ != PST_OK) return st_;      \
  } while (0)

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
  // the tables are rewritten in place: passes still queued with the old ones
  // (this plan's stream) must have finished before the synchronous upload
  if (t.valid) TRY(hip_check(hipStreamSynchronize(pl->stream), "hipStreamSynchronize(tables)"));
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

}  // namespace

extern "C" {

static pst_status nls_check(Plan* pl, const pst_nls_params* p, int nsteps) {
  TRY(need_kind(pl, PST_C2C, "nls_step"));
  if (p == nullptr) return fail(PST_ERR_INVALID, "params is NULL");
  TRY(check_domain(p->d));
  if (!(p->dt != 0.0) || !std::isfinite(p->dt)) return fail(PST_ERR_INVALID, "dt must be finite and nonzero");
  if (!std::isfinite(p->g)) return fail(PST_ERR_INVALID, "g must be finite");
  if (nsteps < 0) return fail(PST_ERR_INVALID, "nsteps must be >= 0");
  return PST_OK;
}

// nsteps Strang steps of the pl->batch fields addressed by psi; fstat (a
// device table of per-field status words, may be NULL) receives
// ST_NONFINITE for a field whose result is not finite.
static pst_status nls_run(Plan* pl, FieldRef psi, const pst_nls_params* p, int nsteps,
                          int* const* fstat = nullptr) {
  if (nsteps == 0) return PST_OK;
  TRY(nls_tables(pl, p));
  if (pl->mixed) {
    // the same sequence of passes on the mixed-radix kernels (plain rows)
    const int nx = pl->nx, ny = pl->ny, B = pl->batch;
    const double pc = p->g * p->dt / ((double)nx * nx);
    const NlsTables& t = pl->nls;
    hipStream_t s = pl->stream;
    auto row = [&](int mode, double pc_, double scale, StatusRef sr) {
      if (mode == 1) prof_begin(pl, PST_PASS_NLS_ROW);
      pst_status r = hip_check(mixed_nls_row(pl->P, pl->mlx, B * ny, ny, psi, mode, pc_, scale, pl->tw_x, s, sr),
                               "nls row");
      if (mode == 1) prof_end(pl);
      return r;
    };
    auto col = [&](const void* ex, const void* ey) {
      prof_begin(pl, PST_PASS_NLS_COL);
      pst_status r = hip_check(mixed_nls_col(pl->P, pl->mly, nx, B, psi, pl->tw_y, ex, ey, s), "nls column");
      prof_end(pl);
      return r;
    };
    TRY(row(0, 0.0, (double)nx, StatusRef()));
    TRY(col(t.ex_half, t.ey_half));
    for (int i = 1; i < nsteps; ++i) {
      TRY(row(1, pc, 1.0, StatusRef()));
      TRY(col(t.ex_full, t.ey_full));
    }
    TRY(row(1, pc, 1.0, StatusRef()));
    TRY(col(t.ex_half, t.ey_half));
    StatusRef sr;
    sr.plan = pl->dstatus;
    sr.field = fstat;
    return row(2, 0.0, 1.0 / nx, sr);
  }
  const int nx = pl->nx, ny = pl->ny, B = pl->batch, W = pl->colvar;
  const int lines = B * ny;
  const double pc = p->g * p->dt / ((double)nx * nx);
  const NlsTables& t = pl->nls;
  hipStream_t s = pl->stream;
  auto row = [&](int mode, double pc_, double scale) {
    if (mode == 1) prof_begin(pl, PST_PASS_NLS_ROW);
    pst_status r = hip_check(nls_row(pl->P, nx, lines, ny, psi, mode, pc_, scale, pl->tw_x, s, StatusRef(),
                                     pl->rowvar),
                             "nls row");
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
  StatusRef sr;
  sr.plan = pl->dstatus;
  sr.field = fstat;
  return hip_check(nls_row(pl->P, nx, lines, ny, psi, 2, 0.0, 1.0 / nx, pl->tw_x, s, sr), "nls exit row");
}

pst_status nls_step(pst_plan pl, void* psi, const pst_nls_params* p, int nsteps) {
  TRY(nls_check(pl, p, nsteps));
  TRY(check_field(psi, "psi"));
  return nls_run(pl, contiguous(psi, (size_t)pl->nx * pl->ny * pl->csize), p, nsteps);
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
    if (pl->mixed) {
      TRY(hip_check(mixed_nls_cq(pl->P, pl->mlx, pl->mly, B, f0, spec, rowp, colp, pl->tw_x, pl->tw_y,
                                 2 * M_PI / p->d.lx, 2 * M_PI / p->d.ly, s),
                    "cq passes"));
    } else {
      TRY(hip_check(nls_cq_row(pl->P, nx, B * ny, f0, spec, rowp, pl->tw_x, s), "cq row"));
      TRY(hip_check(nls_cq_col(pl->P, ny, nx, B, spec, colp, pl->tw_y, 2 * M_PI / p->d.lx,
                               2 * M_PI / p->d.ly, 0, s),
                    "cq column"));
    }
    TRY(hip_check(nls_cq_finish(B, ny, nx, rowp, colp, dxdy, kin, p->g, pl->dres, pl->dstatus, s), "cq finish"));
  } else if (pl->mixed) {
    return fail(PST_ERR_UNSUPPORTED, "conserved_quantities: sine-Gordon and Navier-Stokes need power-of-two sizes");
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
    TRY(hip_check(fft_row_r2c(pl->P, nx, B * ny, ny, contiguous(f0, (size_t)nx * ny * pl->rsize), XH, pl->tw_x, s),
                  "NS cq row"));
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

}  // extern "C"

namespace pst {

pst_status sg_params_check(Plan* pl, const pst_sg_params* p, const char* who) {
  TRY(need_kind(pl, PST_R2C, who));
  if (pl->mixed) return fail(PST_ERR_UNSUPPORTED, "%s: sine-Gordon needs power-of-two sizes", who);
  if (p == nullptr) return fail(PST_ERR_INVALID, "%s: params is NULL", who);
  TRY(check_domain(p->d));
  if (!(p->dt > 0.0) || !std::isfinite(p->dt)) return fail(PST_ERR_INVALID, "%s: dt must be finite and > 0", who);
  return PST_OK;
}

size_t sg_work_bytes(const Plan* pl) {
  const size_t a = ((size_t)pl->batch * pl->ny * (pl->nx / 2 + 1) * pl->csize + 255) & ~(size_t)255;
  return 3 * a;
}

SgWork sg_work_at(const Plan* pl, void* base) {
  const size_t a = sg_work_bytes(pl) / 3;
  char* b = static_cast<char*>(base);
  return SgWork{b, b + a, b + 2 * a};
}

}  // namespace pst

extern "C" {

static pst_status sg_check(Plan* pl, const pst_sg_params* p, const char* who) {
  TRY(sg_params_check(pl, p, who));
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
  const size_t fb = (size_t)nx * ny * pl->rsize;
  void* U = ws_at(pl, pl->off_spec);
  void* S = ws_at(pl, pl->off_spec2);
  void* W = ws_at(pl, pl->off_spec3);
  const double sc = 0.5 / ((double)nx * ny), dt = p->dt;
  hipStream_t s = pl->stream;
  const FieldRef none;
  TRY(hip_check(sg_row(pl->P, 0, nx, lines, ny, nullptr, contiguous(u0, fb), none, 0.0, none, none, none, U, S,
                       pl->tw_x, s),
                "sg entry row"));
  // u^1 - u^0 = iFFT((c1s - 1) U - c2s S) + dt v0, c1s = (1-a)/(1+a), c2s = dt^2/(2(1+a))
  TRY(hip_check(sg_col(pl->P, ny, nx, B, U, S, W, pl->tw_y, 2 * M_PI / p->d.lx, 2 * M_PI / p->d.ly,
                       0.25 * dt * dt, 1.0, 0.5 * dt * dt, sc, col_w(pl, ny), s),
                "sg start column"));
  return hip_check(sg_row(pl->P, 2, nx, lines, ny, W, contiguous(u0, fb), contiguous(v0, fb), dt,
                          contiguous(u_curr, fb), none, contiguous(u_prev, fb), nullptr, nullptr, pl->tw_x, s),
                   "sg start row");
}

}  // extern "C"

// nsteps of the pl->batch field pairs (u_prev, u_curr) in the work arrays w;
// fstat as in nls_run; profile: bracket passes with events when the plan's
// profiling is on.
pst_status pst::sg_run_in(Plan* pl, const SgWork& w, FieldRef u_prev, FieldRef u_curr, const pst_sg_params* p,
                          int nsteps, int* const* fstat, bool profile) {
  if (nsteps == 0) return PST_OK;
  const int nx = pl->nx, ny = pl->ny, B = pl->batch, lines = B * ny;
  void* U = w.U;
  void* S = w.S;
  void* W = w.W;
  const bool prof = profile && pl->prof;
  const double sc = 0.5 / ((double)nx * ny), dt = p->dt;
  const double kx0 = 2 * M_PI / p->d.lx, ky0 = 2 * M_PI / p->d.ly;
  const int Wt = col_w(pl, ny);
  hipStream_t s = pl->stream;
  const FieldRef none;
  auto col = [&]() {
    if (prof) prof_begin(pl, PST_PASS_SG_COL);
    pst_status r = hip_check(sg_col(pl->P, ny, nx, B, U, S, W, pl->tw_y, kx0, ky0, 0.25 * dt * dt, 2.0, dt * dt, sc,
                                    Wt, s),
                             "sg column");
    if (prof) prof_end(pl);
    return r;
  };
  // u_curr holds u^n; u_prev's buffer holds the increment d^n during the call
  TRY(hip_check(sg_row(pl->P, 0, nx, lines, ny, nullptr, u_curr, u_prev, 0.0, none, u_prev, none, U, S, pl->tw_x, s),
                "sg entry row"));
  TRY(col());
  for (int i = 0; i < nsteps - 1; ++i) {
    if (prof) prof_begin(pl, PST_PASS_SG_ROW);
    TRY(hip_check(sg_row(pl->P, 1, nx, lines, ny, W, u_curr, u_prev, 1.0, u_curr, u_prev, none, U, S, pl->tw_x, s),
                  "sg row"));
    if (prof) prof_end(pl);
    TRY(col());
  }
  // last step: u_curr <- u^N, u_prev <- u^{N-1} (the level it replaces)
  StatusRef sr;
  sr.plan = pl->dstatus;
  sr.field = fstat;
  return hip_check(sg_row(pl->P, 2, nx, lines, ny, W, u_curr, u_prev, 1.0, u_curr, none, u_prev, nullptr, nullptr,
                          pl->tw_x, s, sr),
                   "sg final row");
}

// sg_run_in on the plan's workspace.
static pst_status sg_run(Plan* pl, FieldRef u_prev, FieldRef u_curr, const pst_sg_params* p, int nsteps,
                         int* const* fstat = nullptr) {
  const SgWork w{ws_at(pl, pl->off_spec), ws_at(pl, pl->off_spec2), ws_at(pl, pl->off_spec3)};
  return sg_run_in(pl, w, u_prev, u_curr, p, nsteps, fstat, true);
}

extern "C" {

pst_status sg_step(pst_plan pl, void* u_prev, void* u_curr, const pst_sg_params* p, int nsteps) {
  TRY(sg_check(pl, p, "sg_step"));
  TRY(check_field(u_prev, "u_prev"));
  TRY(check_field(u_curr, "u_curr"));
  if (u_prev == u_curr) return fail(PST_ERR_INVALID, "sg_step: u_prev and u_curr must differ");
  if (nsteps < 0) return fail(PST_ERR_INVALID, "nsteps must be >= 0");
  const size_t fb = (size_t)pl->nx * pl->ny * pl->rsize;
  return sg_run(pl, contiguous(u_prev, fb), contiguous(u_curr, fb), p, nsteps);
}

static pst_status ns_check(Plan* pl, const pst_ns_params* p, int nsteps) {
  TRY(need_kind(pl, PST_R2C, "ns_step"));
  if (pl->mixed) return fail(PST_ERR_UNSUPPORTED, "ns_step: Navier-Stokes needs power-of-two sizes");
  if (p == nullptr) return fail(PST_ERR_INVALID, "params is NULL");
  TRY(check_domain(p->d));
  if (!(p->dt > 0.0) || !std::isfinite(p->dt)) return fail(PST_ERR_INVALID, "dt must be finite and > 0");
  if (!(p->nu >= 0.0) || !std::isfinite(p->nu)) return fail(PST_ERR_INVALID, "nu must be finite and >= 0");
  if (!(p->tol >= 0.0)) return fail(PST_ERR_INVALID, "tol must be >= 0");
  if (p->max_iter < 1 || p->max_iter > 10000) return fail(PST_ERR_INVALID, "max_iter must be in [1, 10000]");
  if (p->fixed_iters < 0 || p->fixed_iters > 10000) return fail(PST_ERR_INVALID, "fixed_iters must be in [0, 10000]");
  if (nsteps < 0) return fail(PST_ERR_INVALID, "nsteps must be >= 0");
  return ensure_workspace(pl);
}

// Navier-Stokes steps of the pl->batch vorticity fields addressed by omega,
// as a chunk: entry passes, the steps, exit passes.  Every step queues its
// first iteration and then, gated per field on the device by the
// convergence flags, a fixed number of further ones: exactly fixed_iters in
// fixed-K mode, else the predicted count plus one (ns_guess: the most
// iterations a step took recently).  A field still unconverged after the
// last queued iteration of a step is parked: every later pass of the chunk
// leaves it alone.  The host reads the flags once per chunk (an event on a
// pinned copy); a parked field (rare) is then resumed on its own, with the
// host checking after each iteration until its step converges or reaches
// max_iter, and runs the rest of the chunk the same way.  Results do not
// depend on the prediction, only the number of gated launches does.
struct NsStepper {
  Plan* pl;
  FieldRef omega;
  const pst_ns_params* p;
  int* dev_iters;
  int* const* fstat;
  NsPtrs P;
  NsScalars S;
  int nx, ny, B, lines, h, Wt, fixed;
  int *done, *iters, *park, *park_step, *maxit;
  double* resid;
  double vol, fp_floor;
  int step = 0, target = 1, nsteps = 0;

  NsStepper(Plan* pl_, FieldRef omega_, const pst_ns_params* p_, int* dev_iters_, int* const* fstat_)
      : pl(pl_), omega(omega_), p(p_), dev_iters(dev_iters_), fstat(fstat_) {
    nx = pl->nx;
    ny = pl->ny;
    B = pl->batch;
    lines = B * ny;
    h = nx / 2 + 1;
    Wt = col_w(pl, ny);
    P.Q = ws_at(pl, pl->off_spec);
    P.WN = ws_at(pl, pl->off_spec2);
    P.DK = ws_at(pl, pl->off_spec3);
    P.NH = ws_at(pl, pl->off_spec4);
    P.OUT = ws_at(pl, pl->off_spec4);
    P.D = ws_at(pl, pl->off_hyb);
    P.dstride = (size_t)B * ny * h;
    P.part = static_cast<double*>(ws_at(pl, pl->off_colpart));
    S.kx0 = 2 * M_PI / p->d.lx;
    S.ky0 = 2 * M_PI / p->d.ly;
    S.hnu = 0.5 * p->dt * p->nu;
    S.qdt = 0.5 * p->dt;
    S.nscale = 0.5;
    S.dscale = 1.0 / ((double)nx * ny);
    S.nx = nx;
    S.kx_cut = (nx - 1) / 3;
    S.ky_cut = (ny - 1) / 3;
    // per-field state, B ints each: done, iters, park, park_step, maxit
    done = static_cast<int*>(ws_at(pl, pl->off_nsstate));
    iters = done + B;
    park = done + 2 * B;
    park_step = done + 3 * B;
    maxit = done + 4 * B;
    resid = reinterpret_cast<double*>(static_cast<char*>(ws_at(pl, pl->off_nsstate)) +
                                      ((5 * B * sizeof(int) + 7) & ~(size_t)7));
    vol = (p->d.lx / nx) * (p->d.ly / ny) / ((double)nx * ny);
    const double eps = pl->prec == PST_FP32 ? std::ldexp(1.0, -23) : 0.0;
    fp_floor = (16 * eps) * (16 * eps);
    fixed = p->fixed_iters;
    target = fixed > 0 ? fixed : std::min(std::max(pl->ns_guess, 1) + 1, p->max_iter);
  }
  bool adaptive() const { return fixed <= 0; }
  pst_status row(const int* gate) {
    prof_begin(pl, PST_PASS_NS_ROW);
    pst_status r = hip_check(ns_row(pl->P, nx, lines, ny, P.D, P.dstride, (void*)P.NH, gate, pl->tw_x, pl->stream),
                             "ns row");
    prof_end(pl);
    return r;
  }
  pst_status col(int mode, const int* gate) {
    if (mode == 1 || mode == 2) prof_begin(pl, PST_PASS_NS_COL);
    pst_status r = hip_check(ns_col(pl->P, mode, ny, B, P, S, gate, pl->tw_y, Wt, pl->stream), "ns column");
    if (mode == 1 || mode == 2) prof_end(pl);
    return r;
  }
  pst_status finish(int first, int last) {
    int* iout = dev_iters ? dev_iters + (size_t)step * B : nullptr;
    NsPark pk;
    pk.park = park;
    pk.park_step = park_step;
    pk.maxit = maxit;
    pk.last = last;
    pk.step = step;
    return hip_check(ns_finish(B, h, P.part, vol, p->tol, fp_floor, p->max_iter, fixed, first, done, iters, iout,
                               resid, pl->dstatus, fstat, pk, pl->stream),
                     "ns finish");
  }
  // -- the chunk, queued without host involvement (may be captured) -------
  // entry: no field parked, w^n = rfft2(omega), increment 0, derivatives
  pst_status begin() {
    TRY(hip_check(fill_int(park, 3 * B, 0, pl->stream), "clear ns state"));  // park, park_step, maxit
    TRY(hip_check(fft_row_r2c(pl->P, nx, lines, ny, omega, (void*)P.NH, pl->tw_x, pl->stream), "ns entry row"));
    return col(0, nullptr);
  }
  // one step: the first iteration and target - 1 gated ones; in adaptive
  // mode the last of them parks an unconverged field
  pst_status queue_step() {
    TRY(row(park));
    TRY(col(1, park));
    TRY(finish(1, adaptive() && target == 1));
    for (int i = 2; i <= target; ++i) {
      TRY(row(done));
      TRY(col(2, done));
      TRY(finish(0, adaptive() && i == target));
    }
    ++step;
    return PST_OK;
  }
  // exit: omega = irfft2(w^n + d) for the fields not parked
  pst_status queue_exit() {
    TRY(col(3, park));
    return hip_check(
        fft_row_c2r(pl->P, nx, lines, ny, P.OUT, omega, 1.0 / ((double)nx * ny), pl->tw_x, pl->stream, park),
        "ns exit row");
  }
  pst_status queue_chunk(int k) {
    nsteps = k;
    step = 0;
    TRY(begin());
    for (int i = 0; i < k; ++i) TRY(queue_step());
    return queue_exit();
  }
  // -- host side ------------------------------------------------------------
  pst_status ensure_host(int ints) {
    if (pl->ns_host_n < ints) {
      if (pl->ns_host != nullptr) {
        TRY(hip_check(hipStreamSynchronize(pl->stream), "hipStreamSynchronize"));
        TRY(hip_check(hipHostFree(pl->ns_host), "hipHostFree(ns flags)"));
        pl->ns_host = nullptr;
        pl->ns_host_n = 0;
      }
      TRY(hip_check(hipHostMalloc((void**)&pl->ns_host, ints * sizeof(int), hipHostMallocDefault),
                    "hipHostMalloc(ns flags)"));
      pl->ns_host_n = ints;
    }
    if (pl->ns_ev == nullptr)
      TRY(hip_check(hipEventCreateWithFlags(&pl->ns_ev, hipEventDisableTiming), "hipEventCreate"));
    return PST_OK;
  }
  // copy iters, park, park_step, maxit (contiguous) to the host behind an event
  pst_status request_flags() {
    TRY(hip_check(hipMemcpyAsync(pl->ns_host, iters, 4 * B * sizeof(int), hipMemcpyDeviceToHost, pl->stream),
                  "read ns flags"));
    return hip_check(hipEventRecord(pl->ns_ev, pl->stream), "hipEventRecord");
  }
  // wait for the chunk's flags, update the prediction, resume parked fields
  pst_status complete_chunk() {
    TRY(hip_check(hipEventSynchronize(pl->ns_ev), "hipEventSynchronize"));
    std::vector<int> hostv(pl->ns_host, pl->ns_host + 4 * B);
    const int* h_iters = hostv.data();
    const int* h_park = h_iters + B;
    const int* h_pstep = h_iters + 2 * B;
    const int* h_maxit = h_iters + 3 * B;
    int most = 0;
    for (int f = 0; f < B; ++f) most = std::max(most, h_maxit[f]);
    for (int f = 0; f < B; ++f)
      if (h_park[f]) TRY(resume(f, h_pstep[f], h_iters[f], &most));
    if (most > 0) pl->ns_guess = most;
    return PST_OK;
  }
  // field f stopped in step s of the chunk after `it` iterations: finish that
  // step and the rest of the chunk with the others gated off, checking the
  // convergence flags on the host after each iteration
  pst_status resume(int f, int s, int it, int* most) {
    TRY(hip_check(fill_int(park, B, 1, pl->stream), "gate ns fields"));
    TRY(hip_check(fill_int(park + f, 1, 0, pl->stream), "gate ns fields"));
    TRY(hip_check(fill_int(done, B, 1, pl->stream), "gate ns fields"));
    TRY(hip_check(fill_int(done + f, 1, 0, pl->stream), "gate ns fields"));
    step = s;
    int launched = it;
    // iterate (an unconverged field first iterates, then checks) until
    // done[f] or max_iter
    auto converge = [&](bool iterate_first) -> pst_status {
      for (bool check = !iterate_first;; check = true) {
        if (check) {
          TRY(hip_check(hipMemcpyAsync(pl->ns_host, done + f, sizeof(int), hipMemcpyDeviceToHost, pl->stream),
                        "read ns flag"));
          TRY(hip_check(hipEventRecord(pl->ns_ev, pl->stream), "hipEventRecord"));
          TRY(hip_check(hipEventSynchronize(pl->ns_ev), "hipEventSynchronize"));
          if (pl->ns_host[0] != 0 || launched >= p->max_iter) break;
        }
        TRY(row(done));
        TRY(col(2, done));
        TRY(finish(0, 0));
        ++launched;
      }
      *most = std::max(*most, launched);
      return PST_OK;
    };
    TRY(converge(true));
    for (++step; step < nsteps; ++step) {
      TRY(row(park));
      TRY(col(1, park));
      TRY(finish(1, 0));
      launched = 1;
      TRY(converge(false));
    }
    return queue_exit();
  }
};

static pst_status ns_run(Plan* pl, FieldRef omega, const pst_ns_params* p, int nsteps, int* dev_iters,
                         int* const* fstat = nullptr) {
  if (nsteps == 0) return PST_OK;
  NsStepper st(pl, omega, p, dev_iters, fstat);
  if (st.adaptive()) TRY(st.ensure_host(4 * pl->batch));
  TRY(st.queue_chunk(nsteps));
  if (!st.adaptive()) return PST_OK;
  TRY(st.request_flags());
  return st.complete_chunk();
}

pst_status ns_step(pst_plan pl, void* omega, const pst_ns_params* p, int nsteps, int* dev_iters) {
  TRY(ns_check(pl, p, nsteps));
  TRY(check_field(omega, "omega"));
  return ns_run(pl, contiguous(omega, (size_t)pl->nx * pl->ny * pl->rsize), p, nsteps, dev_iters);
}

}  // extern "C"

// ------------------------------------------------------------ autotune ---
extern "C" pst_status pst_autotune(pst_plan plan, pst_eq eq, int* chosen);
namespace {
std::mutex g_tune_mu;
// (eq, prec, nx, ny) -> (row variant, column variant): every plan of a class
// in the process runs the same variants, so results do not depend on which
// plan (or batch) a field is stepped in
std::map<std::tuple<int, int, int, int>, std::pair<int, int>> g_tuned;
}  // namespace

// Time per launch of `launch`: after one warm-up, a first window of 5
// back-to-back launches sizes the windows to about 1 ms of work (5 to 200
// launches; short launches are otherwise dominated by launch gaps), then
// the best of three such windows (a single window is at the mercy of clock
// ramps and other work on the device).
template <class L>
static pst_status time_launch(Plan* pl, L&& launch, float* ms) {
  hipStream_t s = pl->stream;
  TRY(hip_check(launch(), "autotune warm-up"));
  hipEvent_t a, b;
  TRY(hip_check(hipEventCreate(&a), "hipEventCreate"));
  TRY(hip_check(hipEventCreate(&b), "hipEventCreate"));
  pst_status st = PST_OK;
  auto window = [&](int reps, float* t) {
    st = hip_check(hipEventRecord(a, s), "hipEventRecord");
    for (int i = 0; i < reps && st == PST_OK; ++i) st = hip_check(launch(), "autotune launch");
    if (st == PST_OK) st = hip_check(hipEventRecord(b, s), "hipEventRecord");
    if (st == PST_OK) st = hip_check(hipEventSynchronize(b), "hipEventSynchronize");
    if (st == PST_OK) st = hip_check(hipEventElapsedTime(t, a, b), "hipEventElapsedTime");
  };
  float first = 0.f;
  window(5, &first);
  const int reps = first > 0.f ? std::min(200, std::max(5, (int)std::ceil(5.0f / first))) : 5;
  *ms = 1e30f;
  for (int w = 0; w < 3 && st == PST_OK; ++w) {
    float t = 0.f;
    window(reps, &t);
    if (st == PST_OK && t / reps < *ms) *ms = t / reps;
  }
  (void)hipEventDestroy(a);  // teardown: the timing result is already known
  (void)hipEventDestroy(b);
  return st;
}

// ptab: zeroed propagator stand-in of max(nx, ny) complex entries.  An NLS
// column variant is timed together with the row pass in row variant
// `row` (one step per launch), as the two alternate in a run: a column
// pass timed back to back with itself meets different cache contents.
static pst_status time_col(Plan* pl, pst_eq eq, int w, int row, const void* ptab, float* ms) {
  const int nx = pl->nx, ny = pl->ny, B = pl->batch;
  hipStream_t s = pl->stream;
  auto launch = [&]() -> hipError_t {
    if (eq == PST_NLS) {
      const FieldRef f = contiguous(ws_at(pl, pl->off_spec), (size_t)nx * ny * pl->csize);
      const hipError_t e = nls_row(pl->P, nx, B * ny, ny, f, 1, 1e-9, 1.0, pl->tw_x, s, StatusRef(), row);
      if (e != hipSuccess) return e;
      return nls_col(pl->P, ny, nx, B, f, pl->tw_y, ptab, ptab, w, s);
    }
    if (eq == PST_SG)
      return sg_col(pl->P, ny, nx, B, ws_at(pl, pl->off_spec), ws_at(pl, pl->off_spec2), ws_at(pl, pl->off_spec3),
                    pl->tw_y, 1.0, 1.0, 1e-4, 2.0, 1e-4, 1e-6, w, s);
    NsPtrs P;
    const int h = nx / 2 + 1;
    P.Q = ws_at(pl, pl->off_spec);
    P.WN = ws_at(pl, pl->off_spec2);
    P.DK = ws_at(pl, pl->off_spec3);
    P.NH = ws_at(pl, pl->off_spec4);
    P.OUT = ws_at(pl, pl->off_spec4);
    P.D = ws_at(pl, pl->off_hyb);
    P.dstride = (size_t)B * ny * h;
    P.part = static_cast<double*>(ws_at(pl, pl->off_colpart));
    NsScalars S{2 * M_PI, 2 * M_PI, 5e-7, 5e-4, 0.5, 1.0 / ((double)nx * ny), nx, (nx - 1) / 3, (ny - 1) / 3};
    // the iteration pass (mode 2), which runs several times per step
    return ns_col(pl->P, 2, ny, B, P, S, static_cast<int*>(ws_at(pl, pl->off_nsstate)), pl->tw_y, w, s);
  };
  return time_launch(pl, launch, ms);
}

// The NLS in-place row pass in row variant v on workspace data.
static pst_status time_row(Plan* pl, int v, float* ms) {
  const int nx = pl->nx, ny = pl->ny, B = pl->batch;
  auto launch = [&]() -> hipError_t {
    return nls_row(pl->P, nx, B * ny, ny, contiguous(ws_at(pl, pl->off_spec), (size_t)nx * ny * pl->csize), 1,
                   1e-9, 1.0, pl->tw_x, pl->stream, StatusRef(), v);
  };
  return time_launch(pl, launch, ms);
}

extern "C" pst_status pst_autotune(pst_plan pl, pst_eq eq, int* chosen) {
  if (pl == nullptr) return fail(PST_ERR_INVALID, "plan is NULL");
  if (eq != PST_NLS && eq != PST_SG && eq != PST_NS) return fail(PST_ERR_INVALID, "unknown equation %d", (int)eq);
  TRY(need_kind(pl, eq == PST_NLS ? PST_C2C : PST_R2C, "pst_autotune"));
  if (pl->mixed) {
    // the mixed-radix passes have one configuration
    pl->rowvar = pl->colvar = 0;
    if (chosen) *chosen = 0;
    return PST_OK;
  }
  TRY(ensure_workspace(pl));
  const auto key = std::make_tuple((int)eq, (int)pl->prec, pl->nx, pl->ny);
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) {
      pl->rowvar = it->second.first;
      pl->colvar = it->second.second;
      if (chosen) *chosen = pl->colvar;
      return PST_OK;
    }
  }
  // workspace contents are irrelevant to the timing; start from zeros
  TRY(hip_check(hipMemsetAsync(pl->ws, 0, pl->ws_need, pl->stream), "clear workspace"));
  void* ptab = nullptr;
  const size_t pbytes = (size_t)std::max(pl->nx, pl->ny) * pl->csize;
  TRY(hip_check(hipMalloc(&ptab, pbytes), "hipMalloc(autotune table)"));
  pl->owned.push_back(ptab);
  TRY(hip_check(hipMemsetAsync(ptab, 0, pbytes, pl->stream), "clear autotune table"));
  int best = 0, best_row = 0;
  float best_ms = 1e30f;
  int w, q, sp, r;
  if (eq == PST_NLS) {
    // the row pass first: the column variants are then timed beside it
    for (int v = 0; nls_row_variant_info(pl->P, pl->nx, v, &w, &q, &sp, &r); ++v) {
      float ms = 0.f;
      TRY(time_row(pl, v, &ms));
      if (ms < best_ms) {
        best_ms = ms;
        best_row = v;
      }
    }
    best_ms = 1e30f;
  }
  for (int v = 0; col_variant_info(pl->P, pl->ny, v, eq == PST_NLS, &w, &q, &sp, &r); ++v) {
    float ms = 0.f;
    TRY(time_col(pl, eq, v, best_row, ptab, &ms));
    if (ms < best_ms) {
      best_ms = ms;
      best = v;
    }
  }
  pl->colvar = best;
  pl->rowvar = best_row;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tuned[key] = std::make_pair(best_row, best);
  }
  if (chosen) *chosen = best;
  return PST_OK;
}

// ------------------------------------------------------------ batching ---
// solve_batch groups requests that share (equation, nx, ny, precision,
// parameters).  Each group runs on an internal plan of its size class whose
// capacity is the next power of two of the group size; the callers' fields
// are reached through device pointer tables, so nothing is gathered or
// copied.  Groups are forked onto at most kSideStreams library-owned streams
// (default priority) and joined back on the caller's stream, so size classes
// overlap on the device.  Requests of one group with different step counts
// advance in chunks of the smallest remaining count; a chunk's launch
// sequence is captured into a hipGraph and replayed when the same (fields,
// chunk, parameters) comes back.
namespace {

// Plans are cached per size class and slot: slot s serves the s-th group of
// that class in one call (groups of a class differ only by parameters), so
// the cache holds one plan per class unless calls mix parameter sets.
struct ClassKey {
  int eq, nx, ny, prec, slot;
  bool operator<(const ClassKey& o) const {
    return std::tie(eq, nx, ny, prec, slot) < std::tie(o.eq, o.nx, o.ny, o.prec, o.slot);
  }
};

struct BatchPlan {
  Plan* pl = nullptr;
  void** dtab = nullptr;      // device: cap x {f0, f1, per-field status pointer, caller status pointer}
  int* dfst = nullptr;        // device: per-field status bits
  size_t tab_bytes = 0;
  hipEvent_t last = nullptr;  // recorded on the plan's stream after its last use
  bool used = false;          // last has been recorded
  // chunk schedules seen once, and the graphs of those seen again: a
  // schedule is captured on its second occurrence and replayed from the
  // third on, so one-off schedules (a serving loop's changing mix) never pay
  // for a capture
  std::map<std::vector<uintptr_t>, int> seen;
  std::map<std::vector<uintptr_t>, hipGraphExec_t> graphs;
};
constexpr size_t kMaxGraphs = 64, kMaxSeen = 4096;
// One side stream per hardware queue a process gets by default; further
// groups share them round robin (and run one after another on each).
constexpr int kSideStreams = 4;

std::mutex g_batch_mu;
std::map<ClassKey, BatchPlan> g_batch_plans;
std::vector<hipStream_t> g_side_streams;

size_t params_size(int eq) {
  return eq == PST_NLS ? sizeof(pst_nls_params) : eq == PST_SG ? sizeof(pst_sg_params) : sizeof(pst_ns_params);
}

void destroy_batch_plan(BatchPlan& bp) {
  // Teardown of a cache entry: nothing is left to report a failure to.
  for (auto& g : bp.graphs) (void)hipGraphExecDestroy(g.second);
  bp.graphs.clear();
  if (bp.pl != nullptr) (void)fft2d_destroy(bp.pl);  // synchronises the stream it last ran on
  if (bp.last != nullptr) (void)hipEventDestroy(bp.last);
  bp.pl = nullptr;
  bp.last = nullptr;
}

// The cached plan of (class, slot) with room for cap fields, on stream s:
// s first waits for the plan's previous use (possibly on another stream),
// which still owns the workspace until then.
pst_status batch_plan(const pst_request& r, int slot, int cap, hipStream_t s, BatchPlan** out) {
  ClassKey k{(int)r.eq, r.nx, r.ny, (int)r.prec, slot};
  auto it = g_batch_plans.find(k);
  if (it != g_batch_plans.end() && it->second.pl->batch < cap) {
    destroy_batch_plan(it->second);
    g_batch_plans.erase(it);
    it = g_batch_plans.end();
  }
  if (it == g_batch_plans.end()) {
    BatchPlan bp;
    pst_status st = fft2d_plan(r.nx, r.ny, r.eq == PST_NLS ? PST_C2C : PST_R2C, r.prec, cap, s, &bp.pl);
    if (st == PST_OK) st = ensure_workspace(bp.pl);
    if (st == PST_OK) st = pst_autotune(bp.pl, r.eq, nullptr);
    void* p = nullptr;
    bp.tab_bytes = (size_t)cap * (4 * sizeof(void*) + sizeof(int)) + 256;
    if (st == PST_OK) st = hip_check(hipMalloc(&p, bp.tab_bytes), "hipMalloc(tables)");
    if (st == PST_OK) {
      bp.pl->owned.push_back(p);
      bp.dtab = static_cast<void**>(p);
      bp.dfst = reinterpret_cast<int*>(static_cast<char*>(p) + (size_t)cap * 4 * sizeof(void*));
      st = hip_check(hipEventCreateWithFlags(&bp.last, hipEventDisableTiming), "hipEventCreate");
    }
    if (st != PST_OK) {
      destroy_batch_plan(bp);
      return st;
    }
    it = g_batch_plans.emplace(k, bp).first;
  }
  BatchPlan& bp = it->second;
  if (bp.used && bp.pl->stream != s) TRY(hip_check(hipStreamWaitEvent(s, bp.last, 0), "hipStreamWaitEvent"));
  bp.pl->stream = s;
  *out = &bp;
  return PST_OK;
}

pst_status check_request(const pst_request& r, int i) {
  if (r.eq != PST_NLS && r.eq != PST_SG && r.eq != PST_NS) return fail(PST_ERR_INVALID, "request %d: unknown equation", i);
  if (!size_class(r.nx) || !size_class(r.ny))
    return fail(PST_ERR_INVALID, "request %d: sizes must be 2^a 3^b 5^c in [4, 8192]", i);
  if (r.eq != PST_NLS && (size_class(r.nx) != 1 || size_class(r.ny) != 1))
    return fail(PST_ERR_UNSUPPORTED, "request %d: sine-Gordon and Navier-Stokes need power-of-two sizes", i);
  if (r.prec != PST_FP32 && r.prec != PST_FP64) return fail(PST_ERR_INVALID, "request %d: unknown precision", i);
  if (r.nsteps < 0) return fail(PST_ERR_INVALID, "request %d: nsteps < 0", i);
  if (r.params == nullptr) return fail(PST_ERR_INVALID, "request %d: params is NULL", i);
  pst_status st = check_field(r.f0, "f0");
  if (st == PST_OK && r.eq == PST_SG) st = check_field(r.f1, "f1");
  if (st != PST_OK) return fail(st, "request %d: %s", i, pst_last_error());
  if (r.eq == PST_SG && r.f0 == r.f1) return fail(PST_ERR_INVALID, "request %d: u_prev and u_curr must differ", i);
  if (reinterpret_cast<uintptr_t>(r.dev_status) % alignof(int) != 0)
    return fail(PST_ERR_INVALID, "request %d: dev_status is not int-aligned", i);
  return PST_OK;
}

// Per-request status: the group's per-field bits mapped to a pst_status and
// latched into the caller's word.  A failure already recorded there by an
// earlier call (PST_ERR_NOT_CONVERGED or PST_ERR_NONFINITE) is kept unless
// this call found a worse one; anything else is overwritten.  NONFINITE
// outranks NOT_CONVERGED.
__global__ void k_scatter_status(const int* fst, int* const* dst, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || dst[i] == nullptr) return;
  const int b = fst[i];
  const int now = (b & ST_NONFINITE) ? PST_ERR_NONFINITE : (b & ST_NOT_CONVERGED) ? PST_ERR_NOT_CONVERGED : PST_OK;
  const int old = *dst[i];
  const int kept = (old == PST_ERR_NONFINITE || old == PST_ERR_NOT_CONVERGED) ? old : PST_OK;
  *dst[i] = now > kept ? now : kept;
}

}  // namespace

// Launch a chunk's sequence on the batch plan's stream, or capture it into a
// graph on the second occurrence of its key and replay it from the third.
template <class L>
static pst_status launch_or_replay(BatchPlan& bp, bool capture, const std::vector<uintptr_t>& key, L&& launch) {
  Plan* pl = bp.pl;
  pst_status st = PST_OK;
  auto g = bp.graphs.end();
  if (capture) {
    g = bp.graphs.find(key);
    if (g == bp.graphs.end()) {
      if (bp.seen.size() >= kMaxSeen) bp.seen.clear();
      capture = bp.seen[key]++ > 0;
    }
  }
  if (capture && g == bp.graphs.end() && bp.graphs.size() >= kMaxGraphs) {
    for (auto& e : bp.graphs) (void)hipGraphExecDestroy(e.second);
    bp.graphs.clear();
  }
  if (!capture) {
    st = launch();
  } else {
    if (g == bp.graphs.end()) {
      hipGraph_t graph;
      st = hip_check(hipStreamBeginCapture(pl->stream, hipStreamCaptureModeThreadLocal), "begin capture");
      if (st == PST_OK) {
        pst_status ls = launch();
        hipError_t e = hipStreamEndCapture(pl->stream, &graph);
        st = ls != PST_OK ? ls : hip_check(e, "end capture");
        if (st == PST_OK) {
          hipGraphExec_t ex;
          st = hip_check(hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0), "graph instantiate");
          (void)hipGraphDestroy(graph);  // the instantiated graph does not need it
          if (st == PST_OK) g = bp.graphs.emplace(key, ex).first;
        }
      }
    }
    if (st == PST_OK) st = hip_check(hipGraphLaunch(g->second, pl->stream), "graph launch");
  }
  return st;
}

// One chunk of a fixed-schedule group: every field advances by k steps.
static pst_status run_chunk(BatchPlan& bp, int eq, const void* params, int nf, int k, bool capture,
                            const std::vector<uintptr_t>& key) {
  Plan* pl = bp.pl;
  const int cap = pl->batch;
  pl->batch = nf;  // the chunk's field count; restored on every return
  struct Restore {
    Plan* pl;
    int cap;
    ~Restore() { pl->batch = cap; }
  } restore{pl, cap};
  FieldRef f0, f1;
  f0.table = bp.dtab;
  f1.table = bp.dtab + cap;
  int* const* fst = reinterpret_cast<int* const*>(bp.dtab + 2 * cap);
  // tables are uploaded before any capture (a synchronous copy may not be captured)
  if (eq == PST_NLS) TRY(nls_tables(pl, static_cast<const pst_nls_params*>(params)));
  return launch_or_replay(bp, capture, key, [&]() -> pst_status {
    if (eq == PST_NLS) return nls_run(pl, f0, static_cast<const pst_nls_params*>(params), k, fst);
    if (eq == PST_SG) return sg_run(pl, f0, f1, static_cast<const pst_sg_params*>(params), k, fst);
    return ns_run(pl, f0, static_cast<const pst_ns_params*>(params), k, nullptr, fst);
  });
}

extern "C" pst_status solve_batch(const pst_request* reqs, int n, void* hip_stream) {
  if (n < 0 || (n > 0 && reqs == nullptr)) return fail(PST_ERR_INVALID, "solve_batch: bad request array");
  for (int i = 0; i < n; ++i) TRY(check_request(reqs[i], i));
  std::lock_guard<std::mutex> lock(g_batch_mu);
  hipStream_t caller = reinterpret_cast<hipStream_t>(hip_stream);
  // group by (eq, nx, ny, prec, parameter bytes); slot = index of the group
  // among this call's groups of the same size class
  std::vector<std::vector<int>> groups;
  std::vector<std::vector<unsigned char>> gkeys;
  std::vector<int> slots;
  std::map<std::vector<unsigned char>, int> gidx;
  std::map<std::tuple<int, int, int, int>, int> per_class;
  for (int i = 0; i < n; ++i) {
    const pst_request& r = reqs[i];
    std::vector<unsigned char> key(5 * sizeof(int) + params_size(r.eq));
    int hdr[5] = {(int)r.eq, r.nx, r.ny, (int)r.prec, 0};
    memcpy(key.data(), hdr, sizeof hdr);
    memcpy(key.data() + sizeof hdr, r.params, params_size(r.eq));
    auto it = gidx.find(key);
    if (it == gidx.end()) {
      gidx.emplace(key, (int)groups.size());
      groups.push_back({i});
      gkeys.push_back(key);
      slots.push_back(per_class[std::make_tuple((int)r.eq, r.nx, r.ny, (int)r.prec)]++);
    } else {
      groups[it->second].push_back(i);
    }
  }
  const int nstreams = std::min<int>(kSideStreams, (int)groups.size());
  while ((int)g_side_streams.size() < nstreams) {
    hipStream_t st;
    TRY(hip_check(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "hipStreamCreate"));
    g_side_streams.push_back(st);
  }
  hipEvent_t fork;
  TRY(hip_check(hipEventCreateWithFlags(&fork, hipEventDisableTiming), "hipEventCreate"));
  TRY(hip_check(hipEventRecord(fork, caller), "hipEventRecord"));
  pst_status result = PST_OK;
  for (int i = 0; i < nstreams && result == PST_OK; ++i)
    result = hip_check(hipStreamWaitEvent(g_side_streams[i], fork, 0), "hipStreamWaitEvent");
  // Prepare every group on this thread (plan cache, autotuning, checks).
  struct Job {
    size_t gi;
    BatchPlan* bp;
    bool adaptive;  // NS with a convergence test: host checks once per step
  };
  std::vector<Job> jobs;
  for (size_t gi = 0; gi < groups.size() && result == PST_OK; ++gi) {
    const pst_request& r0 = reqs[groups[gi][0]];
    hipStream_t s = g_side_streams[gi % kSideStreams];
    int cap = 1;
    while (cap < (int)groups[gi].size()) cap <<= 1;
    BatchPlan* bp = nullptr;
    if ((result = batch_plan(r0, slots[gi], cap, s, &bp)) != PST_OK) break;
    // validate the shared parameters through the single-plan checks
    Plan* pl = bp->pl;
    if (r0.eq == PST_NLS) result = nls_check(pl, static_cast<const pst_nls_params*>(r0.params), 0);
    else if (r0.eq == PST_SG) result = sg_check(pl, static_cast<const pst_sg_params*>(r0.params), "solve_batch");
    else result = ns_check(pl, static_cast<const pst_ns_params*>(r0.params), 0);
    const bool adaptive = r0.eq == PST_NS && static_cast<const pst_ns_params*>(r0.params)->fixed_iters <= 0;
    jobs.push_back({gi, bp, adaptive});
    // per-field status bits start clear for this call
    if (result == PST_OK)
      result = hip_check(hipMemsetAsync(bp->dfst, 0, cap * sizeof(int), s), "clear status");
  }
  // table of a chunk's active requests: f0, f1 and status slots
  auto upload_table = [&](size_t ji, const std::vector<int>& act, std::vector<uintptr_t>* key) -> pst_status {
    const std::vector<int>& g = groups[jobs[ji].gi];
    BatchPlan* bp = jobs[ji].bp;
    const int cap = bp->pl->batch;
    std::vector<void*> tab(3 * cap, nullptr);
    for (size_t a = 0; a < act.size(); ++a) {
      const pst_request& r = reqs[g[act[a]]];
      tab[a] = r.f0;
      tab[cap + a] = r.f1;
      tab[2 * cap + a] = bp->dfst + act[a];
      if (key) {
        key->push_back((uintptr_t)r.f0);
        key->push_back((uintptr_t)r.f1);
      }
    }
    return hip_check(hipMemcpyAsync(bp->dtab, tab.data(), tab.size() * sizeof(void*), hipMemcpyHostToDevice,
                                    bp->pl->stream),
                     "upload field table");
  };
  // active requests of a group and the chunk length (smallest remaining count)
  auto next_chunk = [](const std::vector<int>& left, std::vector<int>* act) {
    act->clear();
    int k = 0;
    for (size_t j = 0; j < left.size(); ++j)
      if (left[j] > 0) {
        act->push_back((int)j);
        k = k == 0 ? left[j] : std::min(k, left[j]);
      }
    return k;
  };
  // per-request device status, then the group's join event
  auto close_group = [&](size_t ji) -> pst_status {
    const std::vector<int>& g = groups[jobs[ji].gi];
    BatchPlan* bp = jobs[ji].bp;
    hipStream_t s = bp->pl->stream;
    const int cap = bp->pl->batch;
    std::vector<int*> stp(g.size());
    bool any = false;
    for (size_t j = 0; j < g.size(); ++j) {
      stp[j] = reqs[g[j]].dev_status;
      any = any || stp[j] != nullptr;
    }
    if (any) {
      int** dst = reinterpret_cast<int**>(bp->dtab + 3 * cap);
      TRY(hip_check(hipMemcpyAsync(dst, stp.data(), g.size() * sizeof(int*), hipMemcpyHostToDevice, s),
                    "upload status table"));
      hipLaunchKernelGGL(k_scatter_status, dim3(((int)g.size() + 255) / 256), dim3(256), 0, s, bp->dfst, dst,
                         (int)g.size());
      TRY(hip_check(hipGetLastError(), "status scatter"));
    }
    TRY(hip_check(hipEventRecord(bp->last, s), "hipEventRecord"));
    bp->used = true;
    return PST_OK;
  };
  // the captured launches carry the parameters (time step, domain,
  // coefficients) as kernel arguments: a graph is replayed only for the same
  // parameter bytes
  auto add_params = [&](size_t ji, std::vector<uintptr_t>* key) {
    const std::vector<unsigned char>& pk = gkeys[jobs[ji].gi];
    for (size_t b = 0; b < pk.size(); b += sizeof(uintptr_t)) {
      uintptr_t w = 0;
      memcpy(&w, pk.data() + b, std::min(sizeof(uintptr_t), pk.size() - b));
      key->push_back(w);
    }
  };
  // fixed-schedule group: chunk after chunk, each a graph replay once seen
  auto run_fixed = [&](size_t ji) -> pst_status {
    const std::vector<int>& g = groups[jobs[ji].gi];
    BatchPlan* bp = jobs[ji].bp;
    const pst_request& r0 = reqs[g[0]];
    std::vector<int> left(g.size()), act;
    for (size_t j = 0; j < g.size(); ++j) left[j] = reqs[g[j]].nsteps;
    for (int k; (k = next_chunk(left, &act)) > 0;) {
      std::vector<uintptr_t> key;
      TRY(upload_table(ji, act, &key));
      key.push_back((uintptr_t)k);
      key.push_back((uintptr_t)act.size());
      add_params(ji, &key);
      TRY(run_chunk(*bp, r0.eq, r0.params, (int)act.size(), k, true, key));
      for (int a : act) left[a] -= k;
    }
    return close_group(ji);
  };
  // Fixed-schedule groups first: their launches are asynchronous.  Then the
  // adaptive NS groups, chunk by chunk: a whole chunk of every open group is
  // queued (captured into a graph once its schedule repeats), and only then
  // does the host read each group's flags, once per chunk, resuming the rare
  // field that needed more iterations than were queued.
  std::vector<size_t> adaptive;
  for (size_t ji = 0; ji < jobs.size() && result == PST_OK; ++ji) {
    if (jobs[ji].adaptive) adaptive.push_back(ji);
    else result = run_fixed(ji);
  }
  struct NsGroup {
    size_t ji;
    std::vector<int> left, act;
    int k = 0, cap = 0;
    bool in_chunk = false, closed = false;
    std::unique_ptr<NsStepper> st;
  };
  std::vector<NsGroup> ns(adaptive.size());
  for (size_t a = 0; a < adaptive.size() && result == PST_OK; ++a) {
    NsGroup& q = ns[a];
    q.ji = adaptive[a];
    const std::vector<int>& g = groups[jobs[q.ji].gi];
    q.left.resize(g.size());
    for (size_t j = 0; j < g.size(); ++j) q.left[j] = reqs[g[j]].nsteps;
    q.cap = jobs[q.ji].bp->pl->batch;
  }
  for (bool busy = true; busy && result == PST_OK;) {
    busy = false;
    for (NsGroup& q : ns) {  // queue a chunk of every open group
      if (q.closed || q.in_chunk || result != PST_OK) continue;
      BatchPlan* bp = jobs[q.ji].bp;
      const pst_request& r0 = reqs[groups[jobs[q.ji].gi][0]];
      q.k = next_chunk(q.left, &q.act);
      if (q.k == 0) {
        q.closed = true;
        result = close_group(q.ji);
        continue;
      }
      std::vector<uintptr_t> key;
      if ((result = upload_table(q.ji, q.act, &key)) != PST_OK) break;
      bp->pl->batch = (int)q.act.size();  // the chunk's field count, restored when it completes
      FieldRef f0;
      f0.table = bp->dtab;
      q.st.reset(new NsStepper(bp->pl, f0, static_cast<const pst_ns_params*>(r0.params), nullptr,
                               reinterpret_cast<int* const*>(bp->dtab + 2 * q.cap)));
      if ((result = q.st->ensure_host(4 * q.cap)) != PST_OK) break;
      key.push_back((uintptr_t)q.k);
      key.push_back((uintptr_t)q.act.size());
      key.push_back((uintptr_t)q.st->target);
      add_params(q.ji, &key);
      NsStepper* stp = q.st.get();
      const int k = q.k;
      result = launch_or_replay(*bp, true, key, [&]() -> pst_status { return stp->queue_chunk(k); });
      if (result == PST_OK) result = q.st->request_flags();
      q.in_chunk = true;
      busy = true;
    }
    for (NsGroup& q : ns) {  // wait for each chunk's flags
      if (!q.in_chunk || result != PST_OK) continue;
      result = q.st->complete_chunk();
      jobs[q.ji].bp->pl->batch = q.cap;
      for (int a : q.act) q.left[a] -= q.k;
      q.in_chunk = false;
      busy = true;
    }
  }
  for (NsGroup& q : ns) jobs[q.ji].bp->pl->batch = q.cap;  // also after an error
  for (const Job& j : jobs) {
    if (!j.bp->used) continue;
    pst_status w = hip_check(hipStreamWaitEvent(caller, j.bp->last, 0), "join wait");
    if (result == PST_OK) result = w;
  }
  (void)hipEventDestroy(fork);
  return result;
}

extern "C" pst_status pst_batch_cache_bytes(size_t* bytes) {
  if (bytes == nullptr) return fail(PST_ERR_INVALID, "bytes is NULL");
  std::lock_guard<std::mutex> lock(g_batch_mu);
  size_t tot = 0;
  for (auto& e : g_batch_plans) {
    const Plan* pl = e.second.pl;
    tot += pl->ws_need + e.second.tab_bytes + 256 + (size_t)pl->batch * 8 * sizeof(double);
    tot += (size_t)(pl->nx + pl->ny) * pl->csize;  // twiddles
    if (pl->kind == PST_C2C) tot += 2 * (size_t)(pl->nx + pl->ny) * pl->csize;  // propagator tables
  }
  *bytes = tot;
  return PST_OK;
}

extern "C" pst_status pst_batch_cache_release(void) {
  std::lock_guard<std::mutex> lock(g_batch_mu);
  for (auto& e : g_batch_plans) destroy_batch_plan(e.second);
  g_batch_plans.clear();
  return PST_OK;
}
