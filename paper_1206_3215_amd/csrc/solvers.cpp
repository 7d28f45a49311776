// Solver drivers of the C ABI: launch sequences of the fused passes.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <vector>

#include "launch.hpp"
#include "runtime.hpp"

using namespace pst;

namespace {

// exp(-i k^2 tau) for the n wavenumbers of a period, in double.
std::vector<std::complex<double>> propagator(int n, double length, double tau) {
  std::vector<std::complex<double>> e(n);
  for (int m = 0; m < n; ++m) {
    const double k = wavenumber(m, n, length);
    const double ph = k * k * tau;
    e[m] = std::complex<double>(std::cos(ph), -std::sin(ph));
  }
  return e;
}

pst_status nls_tables(Plan* pl, const pst_nls_params* p) {
  NlsTables& t = pl->nls;
  if (t.valid && t.dt == p->dt && t.lx == p->d.lx && t.ly == p->d.ly) return PST_OK;
  // 1/(nx ny) is a power of two, so scaling the rounded entries is exact.
  const double inv = 1.0 / ((double)pl->nx * pl->ny);
  pst_status st = upload_complex(pl, propagator(pl->nx, p->d.lx, 0.5 * p->dt), &t.ex_half, true, 1.0);
  if (st == PST_OK) st = upload_complex(pl, propagator(pl->nx, p->d.lx, p->dt), &t.ex_full, true, 1.0);
  if (st == PST_OK) st = upload_complex(pl, propagator(pl->ny, p->d.ly, 0.5 * p->dt), &t.ey_half, true, inv);
  if (st == PST_OK) st = upload_complex(pl, propagator(pl->ny, p->d.ly, p->dt), &t.ey_full, true, inv);
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
  } else if (eq == PST_SG || eq == PST_NS) {
    (void)f1;
    return fail(PST_ERR_UNSUPPORTED, "conserved_quantities: equation not available yet");
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

pst_status sg_start(pst_plan pl, const void*, const void*, void*, void*, const pst_sg_params*) {
  TRY(need_kind(pl, PST_R2C, "sg_start"));
  return fail(PST_ERR_UNSUPPORTED, "sg_start: not available yet");
}

pst_status sg_step(pst_plan pl, void*, void*, const pst_sg_params*, int) {
  TRY(need_kind(pl, PST_R2C, "sg_step"));
  return fail(PST_ERR_UNSUPPORTED, "sg_step: not available yet");
}

pst_status ns_step(pst_plan pl, void*, const pst_ns_params*, int, int*) {
  TRY(need_kind(pl, PST_R2C, "ns_step"));
  return fail(PST_ERR_UNSUPPORTED, "ns_step: not available yet");
}

pst_status solve_batch(const pst_request*, int, void*) {
  return fail(PST_ERR_UNSUPPORTED, "solve_batch: not available yet");
}

}  // extern "C"
