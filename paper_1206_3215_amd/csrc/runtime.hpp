// Internal definitions shared by the host-side translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <string>
#include <vector>

#include "launch.hpp"
#include "pst.h"

// Cached NLS propagator tables for one (dt, domain).
struct NlsTables {
  bool valid = false;
  double dt = 0, lx = 0, ly = 0;
  void* ex_half = nullptr;  // exp(-i kx^2 dt/2) - 1
  void* ex_full = nullptr;  // exp(-i kx^2 dt) - 1
  void* ey_half = nullptr;  // exp(-i ky^2 dt/2) - 1
  void* ey_full = nullptr;  // exp(-i ky^2 dt) - 1
};

struct pst_plan_s {
  int nx = 0, ny = 0, batch = 1;
  pst_kind kind = PST_C2C;
  pst_prec prec = PST_FP32;
  pst::Prec P = pst::P32;
  hipStream_t stream = nullptr;
  int device = 0;
  size_t csize = 8, rsize = 4;  // bytes per complex / real element
  bool mixed = false;           // nx or ny not a power of two: mixed-radix passes
  pst::MixedLine mlx, mly;      // their stage lists (tw_x, tw_y then hold mixed-radix tables)
  int colvar = 0;               // column tile variant for length ny
  int rowvar = 0;               // row variant of the NLS in-place row pass (length nx)
  void* tw_x = nullptr;         // twiddles of the x lines (length nx)
  void* tw_y = nullptr;         // twiddles of the y lines (length ny)
  int* dstatus = nullptr;       // latched device status bits
  double* dres = nullptr;       // batch*8 doubles of reduction results
  std::vector<void*> owned;     // device allocations released with the plan
  // workspace
  void* ws = nullptr;
  bool ws_owned = false;
  size_t ws_need = 0;
  size_t off_spec = 0, off_spec2 = 0, off_spec3 = 0, off_spec4 = 0, off_hyb = 0, off_rowpart = 0,
         off_colpart = 0, off_nsstate = 0;
  int ns_guess = 3;  // predicted fixed-point iterations for the next step
  int* ns_host = nullptr;       // pinned host copy of the NS done/iteration flags
  int ns_host_n = 0;            // ints ns_host holds (2 per field of the largest batch seen)
  hipEvent_t ns_ev = nullptr;   // recorded after the flags' device-to-host copy
  NlsTables nls;
  // per-pass timing (pst_profile_enable)
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_rec;
};

namespace pst {

typedef pst_plan_s Plan;

pst_status fail(pst_status st, const char* fmt, ...);
pst_status hip_check(hipError_t e, const char* what);
pst_status upload_complex(Plan* pl, const std::vector<std::complex<double>>& h, void** dptr, bool unit,
                          double scale);
pst_status check_domain(const pst_domain& d);
pst_status check_field(const void* p, const char* name);
// 1: a power of two in [4, 8192]; 2: another 2^a 3^b 5^c in [4, 8192]; 0: neither.
int size_class(int n);
pst_status ensure_workspace(Plan* pl);
double wavenumber(int m, int n, double length);

// Bracket one pass launch with events when profiling is on.
void prof_begin(Plan* pl, int pass);
void prof_end(Plan* pl);

inline void* ws_at(Plan* pl, size_t off) { return static_cast<char*>(pl->ws) + off; }

// Sine-Gordon steps (solvers.cpp) on work arrays the caller chooses: the
// half spectra U, S and W, each [batch][ny][nx/2+1] complex of the plan's
// precision.  sg_params_check validates without touching the workspace;
// sg_work_bytes is the size of the three arrays (each 256-byte aligned) and
// sg_work_at lays them out from base.
struct SgWork {
  void* U;
  void* S;
  void* W;
};
pst_status sg_params_check(Plan* pl, const pst_sg_params* p, const char* who);
size_t sg_work_bytes(const Plan* pl);
SgWork sg_work_at(const Plan* pl, void* base);
pst_status sg_run_in(Plan* pl, const SgWork& w, FieldRef u_prev, FieldRef u_curr, const pst_sg_params* p,
                     int nsteps, int* const* fstat, bool profile);
inline int col_w(Plan* pl, int n) { return n == pl->ny ? pl->colvar : 0; }

}  // namespace pst
