// C ABI of libhgks (declared in include/hgks.h): parameter checks, workspace
// carving and the sequencing of the two-stage step (Eq. (two-stage) of Sec. 2.1)
// on the caller's stream.  The library allocates no device memory.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/hgks.h"
#include "internal.hpp"

using namespace hgks;

// Workspace of hgks_step_static: one file-scope device array, a copy of which
// every device the library runs on holds for the life of the process.  Host
// code never uses the array's name as an address (in host code it names a
// host-side stand-in); it uses the device address hipGetSymbolAddress returns,
// taken once per device with that device current (static_workspace below).
static __device__ __align__(256) char scratch[HGKS_STATIC_WORKSPACE_BYTES];

struct hgks_handle {
  hgks_params p;
  Geo geo;
  double* q;            // caller's state
  hipStream_t stream;
  char* ws;
  size_t ws_bytes;
  // workspace carve
  Ctrl* ctrl;
  double* qs;           // Q* / Q^{n+1} ping-pong partner of q
  double* rr;           // R = Q^n + dt L + dt^2/6 dL
  void* fl;             // face fluxes of the three directions [3][10][N], FP64 or FP32
  double* diag_part;    // block partials of the diagnostics
  double* diag_out;     // derived diagnostics [HGKS_NDIAG]
  double* speed_part;   // block maxima of the CFL speed
  double* lam_star;     // adjoint of Q* (step adjoint)
  double* mflux;        // constant bulk momentum: stage-2 block sums, then the step's force
  long long steps_done; // steps advanced over the handle's lifetime
  int failed_step;
  // optional per-kernel timing
  bool profiling;
  std::vector<hipEvent_t> events;          // pool, two per recorded launch
  std::vector<int> pending_class;          // class of each recorded launch in this call
  double prof_ms[HGKS_KCLASS_COUNT];
  long long prof_count[HGKS_KCLASS_COUNT];
};

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  size_t ctrl, qs, rr, fl, diag_part, diag_out, speed_part, lam_star, ymet, fwall, mflux, total;
};

Layout layout_for(const hgks_params* p) {
  const long long N = (long long)p->nx * p->ny * p->nz;
  const size_t tf = p->precision == HGKS_PREC_F32FLUX ? sizeof(float) : sizeof(double);
  Layout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  L.ctrl = take(sizeof(Ctrl));
  L.qs = take(sizeof(double) * 5 * N);
  L.rr = take(sizeof(double) * 5 * N);
  L.fl = take(tf * 30 * N);
  L.diag_part = take(sizeof(double) * diag_partial_doubles());
  L.diag_out = take(sizeof(double) * 64);
  L.speed_part = take(sizeof(double) * size_t((N + 255) / 256));
  L.lam_star = take(sizeof(double) * 5 * N);
  // channel: metric tables of the stretched y mesh, fluxes of the bottom wall faces
  L.ymet = take(p->stretch_b > 0.0 ? sizeof(double) * (size_t(kYmTableDoubles) * p->ny + 1) : 0);
  L.fwall = take(p->bc_y == HGKS_BC_WALL_ISOTHERMAL ? tf * 10 * size_t(p->nx) * p->nz : 0);
  // constant bulk momentum: three block sums per stage-2 block, then the force
  L.mflux = take(p->bulk_momentum > 0.0 ? sizeof(double) * (3 * size_t((N + 255) / 256) + 1) : 0);
  L.total = off;
  return L;
}

// Metric tables of the tanh mesh y = tanh(b (eta / (1.5 pi) - 1)) / tanh b on
// eta in [0, 3 pi] (Sec. 3.3), in the layout the device reads (ym_* accessors).
std::vector<double> metric_tables(int ny, double b) {
  const double pi = 3.14159265358979323846;
  const double deta = 3.0 * pi / ny;
  const double gs = 1.0 / (2.0 * std::sqrt(3.0));
  auto ymap = [&](double eta) { return std::tanh(b * (eta / (1.5 * pi) - 1.0)) / std::tanh(b); };
  auto dymap = [&](double eta) {
    double t = std::tanh(b * (eta / (1.5 * pi) - 1.0));
    return b / (1.5 * pi) * (1.0 - t * t) / std::tanh(b);
  };
  std::vector<double> t(size_t(kYmTableDoubles) * ny + 1);
  for (int j = 0; j < ny; ++j) {
    const double dy = ymap((j + 1) * deta) - ymap(j * deta);
    t[j] = 1.0 / dy;
    t[ny + j] = dy;
    for (int m = 0; m < 2; ++m) {
      const double eta = (j + 0.5 + (m == 0 ? -gs : gs)) * deta;
      const double d = dymap(eta);
      t[3 * ny + 1 + 2 * j + m] = 1.0 / (d * deta);
      t[5 * ny + 1 + 2 * j + m] = d * deta / dy;
    }
  }
  for (int f = 0; f <= ny; ++f) t[2 * ny + f] = 1.0 / (dymap(f * deta) * deta);
  return t;
}

int validate(const hgks_params* p) {
  if (!p) return HGKS_E_INVALID_ARG;
  const int minp = 6;
  if (p->nx < minp || p->ny < minp || p->nz < minp) return HGKS_E_INVALID_ARG;
  if (!(p->lx > 0) || !(p->ly > 0) || !(p->lz > 0)) return HGKS_E_INVALID_ARG;
  if (!(p->gamma > 1.0) || !(p->prandtl > 0.0) || !(p->mu_ref >= 0.0) || !(p->cfl > 0.0)) return HGKS_E_INVALID_ARG;
  if (p->mu_exp != 0.0 && !(p->T_ref > 0.0)) return HGKS_E_INVALID_ARG;
  if (p->mode != HGKS_MODE_SMOOTH && p->mode != HGKS_MODE_WENOZ && p->mode != HGKS_MODE_WENOZ_CHAR)
    return HGKS_E_INVALID_ARG;
  if (p->precision != HGKS_PREC_F64 && p->precision != HGKS_PREC_F32FLUX) return HGKS_E_INVALID_ARG;
  if (p->bc_y != HGKS_BC_PERIODIC && p->bc_y != HGKS_BC_WALL_ISOTHERMAL) return HGKS_E_INVALID_ARG;
  long long N = (long long)p->nx * p->ny * p->nz;
  if (N > (1LL << 31) - 1) return HGKS_E_INVALID_ARG;  // 32-bit cell counts in the launch grids
  if (p->mode != HGKS_MODE_SMOOTH) {
    if (!(p->weno_eps > 0.0) || p->weno_p < 1 || p->weno_p > 4 || !(p->c_art >= 0.0)) return HGKS_E_INVALID_ARG;
  }
  if (!(p->stretch_b >= 0.0)) return HGKS_E_INVALID_ARG;
  if (!(p->bulk_momentum >= 0.0) || !std::isfinite(p->bulk_momentum)) return HGKS_E_INVALID_ARG;
  if (p->bulk_momentum > 0.0 && p->body_force_x != 0.0) return HGKS_E_INVALID_ARG;
  if (p->bc_y == HGKS_BC_WALL_ISOTHERMAL && !(p->T_wall > 0.0)) return HGKS_E_INVALID_ARG;
  // the stretched mesh is the channel's wall-normal mesh; walls and stretching
  // are implemented for the smooth mode
  if (p->stretch_b > 0.0 && p->bc_y != HGKS_BC_WALL_ISOTHERMAL) return HGKS_E_UNSUPPORTED;
  if (p->mode != HGKS_MODE_SMOOTH && (p->bc_y != HGKS_BC_PERIODIC || p->stretch_b > 0.0)) return HGKS_E_UNSUPPORTED;
  return HGKS_OK;
}

Geo make_geo(const hgks_params* p) {
  Geo g;
  g.n[0] = p->nx;
  g.n[1] = p->ny;
  g.n[2] = p->nz;
  g.N = (long long)p->nx * p->ny * p->nz;
  g.stride[0] = 1;
  g.stride[1] = p->nx;
  g.stride[2] = (long long)p->nx * p->ny;
  g.h[0] = p->lx / p->nx;
  // stretched y: h[1] is the uniform spacing of eta on [0, 3 pi]
  g.h[1] = p->stretch_b > 0.0 ? 3.0 * 3.14159265358979323846 / p->ny : p->ly / p->ny;
  g.h[2] = p->lz / p->nz;
  for (int a = 0; a < 3; ++a) g.inv_h[a] = 1.0 / g.h[a];
  g.gamma = p->gamma;
  g.gm1 = p->gamma - 1.0;
  g.inv_gm1 = 1.0 / g.gm1;
  g.cp = p->gamma / (p->gamma - 1.0);
  g.inv_pr = 1.0 / p->prandtl;
  g.pr_fix = 1.0 / p->prandtl - 1.0;
  g.K = (5.0 - 3.0 * p->gamma) / (p->gamma - 1.0);
  g.mub_m23 = 2.0 * g.K / (3.0 * (g.K + 3.0)) - 2.0 / 3.0;
  g.mu_ref = p->mu_ref;
  g.T_ref = p->T_ref;
  g.mu_exp = p->mu_exp;
  g.cfl = p->cfl;
  g.weno_eps = p->weno_eps;
  g.weno_p = p->weno_p;
  g.c_art = p->c_art;
  g.wall_y = p->bc_y == HGKS_BC_WALL_ISOTHERMAL;
  g.stretch_y = p->stretch_b > 0.0;
  g.T_wall = p->T_wall;
  g.fx = p->body_force_x;
  g.ym = nullptr;
  g.fwall = nullptr;
  g.rho_ref = 1.0;
  g.p_ref = 1.0;
  g.E_ref = g.p_ref * g.inv_gm1;
  g.H_ref = g.gamma * g.p_ref * g.inv_gm1;
  return g;
}

// Reference state of the flux arithmetic: density and pressure of cell 0 of the
// initial state, with zero velocity.
void set_reference(Geo& g, double rho, double p) {
  g.rho_ref = rho;
  g.p_ref = p;
  g.E_ref = p * g.inv_gm1;
  g.H_ref = g.gamma * p * g.inv_gm1;
}

bool f32(const hgks_handle* h) { return h->p.precision == HGKS_PREC_F32FLUX; }

int hip_status(hipError_t e) { return e == hipSuccess ? HGKS_OK : HGKS_E_DEVICE; }

// Timing brackets (no-ops unless profiling is enabled).
bool prof_begin(hgks_handle* h, int cls) {
  if (!h->profiling) return false;
  size_t k = h->pending_class.size();
  while (h->events.size() < 2 * (k + 1)) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return false;
    h->events.push_back(e);
  }
  h->pending_class.push_back(cls);
  (void)hipEventRecord(h->events[2 * k], h->stream);
  return true;
}
void prof_end(hgks_handle* h, bool on) {
  if (on) (void)hipEventRecord(h->events[2 * (h->pending_class.size() - 1) + 1], h->stream);
}
// after a stream synchronization: fold the recorded launches into the totals
void prof_collect(hgks_handle* h) {
  for (size_t k = 0; k < h->pending_class.size(); ++k) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, h->events[2 * k], h->events[2 * k + 1]) == hipSuccess) {
      h->prof_ms[h->pending_class[k]] += ms;
      h->prof_count[h->pending_class[k]] += 1;
    }
  }
  h->pending_class.clear();
}

template <typename TF>
TF* fl_dir(hgks_handle* h, int d) {
  return static_cast<TF*>(h->fl) + (size_t)d * 10 * h->geo.N;
}

// face fluxes of direction d of state src into the face-flux array fl, by the
// kernel of the handle's mode (stage 2: time derivative only)
template <typename TF>
void mode_flux(hgks_handle* h, int d, bool stage2, const double* src, TF* fl, const int* stop) {
  switch (h->p.mode) {
    case HGKS_MODE_WENOZ: launch_flux_z(h->geo, d, stage2, src, fl, stop, &h->ctrl->dt, h->stream); break;
    case HGKS_MODE_WENOZ_CHAR: launch_flux_zc(h->geo, d, stage2, src, fl, stop, &h->ctrl->dt, h->stream); break;
    default: launch_flux_fused(h->geo, d, stage2, src, fl, stop, h->stream);
  }
}

// fluxes of all three directions of state src into h->fl (stage 2: time derivative only)
void all_fluxes(hgks_handle* h, const double* src, bool stage2, const int* stop) {
  for (int d = 0; d < 3; ++d) {
    bool on = prof_begin(h, stage2 ? HGKS_KCLASS_FLUX_STAGE2 : HGKS_KCLASS_FLUX_STAGE1);
    if (f32(h)) mode_flux(h, d, stage2, src, fl_dir<float>(h, d), stop);
    else mode_flux(h, d, stage2, src, fl_dir<double>(h, d), stop);
    prof_end(h, on);
  }
}

// scratch of the smooth-mode operator VJP: 10 N doubles of face-field cotangents
// in the face-flux arrays, which the step adjoint no longer needs once Q* is formed
// (30 N values of the flux type: 240 B per cell in FP64, 120 in the FP32 form)
double* vjp_scratch(hgks_handle* h) { return reinterpret_cast<double*>(h->fl); }

// adjoint of the face fluxes of all three directions (one timed launch pair each)
void operator_vjp(hgks_handle* h, const double* q, const double* A, const double* B, double cLA, double cLB,
                  double cDA, double cDB, double* lam) {
  for (int d = 0; d < 3; ++d) {
    bool on = prof_begin(h, HGKS_KCLASS_OPERATOR_VJP);
    if (h->p.mode == HGKS_MODE_WENOZ)
      launch_operator_vjp_z(h->geo, d, q, A, B, cLA, cLB, cDA, cDB, &h->ctrl->dt, lam, h->stream);
    else
      launch_operator_vjp(h->geo, d, f32(h), q, A, B, cLA, cLB, cDA, cDB, vjp_scratch(h), lam, h->stream);
    prof_end(h, on);
  }
}

void stage1(hgks_handle* h, const double* cur, double* other, int step) {
  if (f32(h))
    launch_stage1(h->geo, cur, fl_dir<float>(h, 0), other, h->rr, h->ctrl, step, h->stream);
  else
    launch_stage1(h->geo, cur, fl_dir<double>(h, 0), other, h->rr, h->ctrl, step, h->stream);
}

void stage2(hgks_handle* h, const double* cur, double* other, int step) {
  // with constant bulk momentum the stage-2 kernel leaves the force out and writes
  // block sums instead of speed maxima; the force kernels finish the step
  if (f32(h))
    launch_stage2(h->geo, h->rr, fl_dir<float>(h, 0), cur, other, h->ctrl, h->speed_part, h->mflux, step,
                  h->stream);
  else
    launch_stage2(h->geo, h->rr, fl_dir<double>(h, 0), cur, other, h->ctrl, h->speed_part, h->mflux, step,
                  h->stream);
  if (h->mflux) launch_bulk_force(h->geo, cur, other, h->ctrl, h->mflux, h->p.bulk_momentum, h->speed_part, step,
                                  h->stream);
}

constexpr size_t kStaticWorkspaceBytes = HGKS_STATIC_WORKSPACE_BYTES;
constexpr int kMaxDevices = 64;

// The calling thread's current device's copy of scratch, or nullptr if the
// runtime cannot provide it.
void* static_workspace() {
  static std::once_flag once[kMaxDevices];
  static void* addr[kMaxDevices];
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::call_once(once[dev], [dev] {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) == hipSuccess) addr[dev] = ptr;
  });
  return addr[dev];
}

}  // namespace

extern "C" {

int hgks_step_static(const hgks_params* p, double* q, int32_t nsteps, double dt, double* dt_taken,
                     void* hip_stream) {
  int v = validate(p);
  if (v != HGKS_OK) return v;
  if (!q || nsteps < 0) return HGKS_E_INVALID_ARG;
  if (layout_for(p).total > kStaticWorkspaceBytes) return HGKS_E_WORKSPACE;
  void* ws = static_workspace();
  if (!ws) return HGKS_E_DEVICE;
  // hgks_init clears the control block; every other part of the workspace the
  // step reads is written earlier in the same call
  hgks_handle* h = nullptr;
  int st = hgks_init(p, q, ws, kStaticWorkspaceBytes, hip_stream, &h);
  if (st != HGKS_OK) return st;
  st = hgks_step(h, nsteps, dt, dt_taken);
  hgks_destroy(h);
  return st;
}

size_t hgks_workspace_bytes(const hgks_params* p) {
  int v = validate(p);
  if (v != HGKS_OK) return 0;
  return layout_for(p).total;
}

int hgks_init(const hgks_params* p, double* q, void* workspace, size_t ws_bytes, void* hip_stream,
              hgks_handle** out) {
  if (!out) return HGKS_E_INVALID_ARG;
  *out = nullptr;
  int v = validate(p);
  if (v != HGKS_OK) return v;
  if (!q) return HGKS_E_INVALID_ARG;
  const long long N = (long long)p->nx * p->ny * p->nz;
  Layout L = layout_for(p);
  if (!workspace || ws_bytes < L.total || (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0)
    return HGKS_E_WORKSPACE;
  hgks_handle* h = new (std::nothrow) hgks_handle;
  if (!h) return HGKS_E_INVALID_ARG;
  h->p = *p;
  h->geo = make_geo(p);
  h->q = q;
  h->stream = reinterpret_cast<hipStream_t>(hip_stream);
  h->ws = static_cast<char*>(workspace);
  h->ws_bytes = ws_bytes;
  h->ctrl = reinterpret_cast<Ctrl*>(h->ws + L.ctrl);
  h->qs = reinterpret_cast<double*>(h->ws + L.qs);
  h->rr = reinterpret_cast<double*>(h->ws + L.rr);
  h->fl = h->ws + L.fl;
  h->diag_part = reinterpret_cast<double*>(h->ws + L.diag_part);
  h->diag_out = reinterpret_cast<double*>(h->ws + L.diag_out);
  h->speed_part = reinterpret_cast<double*>(h->ws + L.speed_part);
  h->lam_star = reinterpret_cast<double*>(h->ws + L.lam_star);
  if (h->geo.stretch_y) h->geo.ym = reinterpret_cast<const double*>(h->ws + L.ymet);
  if (h->geo.wall_y) h->geo.fwall = h->ws + L.fwall;
  h->mflux = p->bulk_momentum > 0.0 ? reinterpret_cast<double*>(h->ws + L.mflux) : nullptr;
  h->steps_done = 0;
  h->failed_step = -1;
  h->profiling = false;
  for (int k = 0; k < HGKS_KCLASS_COUNT; ++k) { h->prof_ms[k] = 0.0; h->prof_count[k] = 0; }
  launch_reset_ctrl(h->ctrl, h->stream);
  std::vector<double> tables;  // kept alive until the stream synchronization below
  if (h->geo.stretch_y) {
    tables = metric_tables(p->ny, p->stretch_b);
    if (hipMemcpyAsync(h->ws + L.ymet, tables.data(), sizeof(double) * tables.size(), hipMemcpyHostToDevice,
                       h->stream) != hipSuccess) {
      delete h;
      return HGKS_E_DEVICE;
    }
  }
  double c0[5];
  for (int k = 0; k < 5; ++k) {
    if (hipMemcpyAsync(&c0[k], q + (size_t)k * N, sizeof(double), hipMemcpyDeviceToHost, h->stream) != hipSuccess) {
      delete h;
      return HGKS_E_DEVICE;
    }
  }
  if (hipStreamSynchronize(h->stream) != hipSuccess || hipGetLastError() != hipSuccess) {
    delete h;
    return HGKS_E_DEVICE;
  }
  const double p0 = h->geo.gm1 * (c0[4] - 0.5 * (c0[1] * c0[1] + c0[2] * c0[2] + c0[3] * c0[3]) / c0[0]);
  if (!(c0[0] > 0.0) || !(p0 > 0.0) || !std::isfinite(p0)) {
    delete h;
    return HGKS_E_NONPHYSICAL;
  }
  set_reference(h->geo, c0[0], p0);
  *out = h;
  return HGKS_OK;
}

int hgks_step(hgks_handle* h, int32_t nsteps, double dt, double* dt_taken) {
  if (!h || nsteps < 0) return HGKS_E_INVALID_ARG;
  if (nsteps == 0) return HGKS_OK;
  if (!(dt > 0.0)) dt = 0.0;
  const Geo& g = h->geo;
  hipStream_t st = h->stream;
  const long long s0 = h->steps_done;
  int done = 0;
  while (done < nsteps) {
    const int chunk = (nsteps - done) < kDtHist ? (nsteps - done) : kDtHist;
    launch_reset_ctrl(h->ctrl, st);
    launch_check_state(g, h->q, h->ctrl, h->speed_part, int(s0 + done) - 1, st);
    double* cur = h->q;
    double* other = h->qs;
    for (int s = 0; s < chunk; ++s) {
      const int step = int(s0 + done + s);
      bool on = prof_begin(h, HGKS_KCLASS_DT);
      launch_dt(g, h->speed_part, h->ctrl, dt, s, st);
      prof_end(h, on);
      all_fluxes(h, cur, false, &h->ctrl->flag);
      on = prof_begin(h, HGKS_KCLASS_STAGE1);
      stage1(h, cur, other, step);
      prof_end(h, on);
      all_fluxes(h, other, true, &h->ctrl->flag);
      on = prof_begin(h, HGKS_KCLASS_STAGE2);
      stage2(h, cur, other, step);
      prof_end(h, on);
      double* t = cur;
      cur = other;
      other = t;
    }
    if (hipGetLastError() != hipSuccess) return HGKS_E_DEVICE;
    Ctrl host;
    if (hipMemcpyAsync(&host, h->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st) != hipSuccess)
      return HGKS_E_DEVICE;
    if (hipStreamSynchronize(st) != hipSuccess) return HGKS_E_DEVICE;
    prof_collect(h);
    if (host.flag) {
      // the last good state is the one the failing step started from
      const long long local = (long long)host.fail_step - (s0 + done);
      if (local >= 0 && (local & 1)) {
        launch_copy(h->qs, h->q, 5 * g.N, st);
        if (hipStreamSynchronize(st) != hipSuccess) return HGKS_E_DEVICE;
      }
      if (dt_taken && local > 0)
        for (long long s = 0; s < local; ++s) dt_taken[done + s] = host.dt_hist[s];
      h->failed_step = host.fail_step;
      h->steps_done = local > 0 ? s0 + done + local : s0 + done;
      return HGKS_E_NONPHYSICAL;
    }
    if (cur != h->q) launch_copy(cur, h->q, 5 * g.N, st);
    if (dt_taken)
      for (int s = 0; s < chunk; ++s) dt_taken[done + s] = host.dt_hist[s];
    done += chunk;
  }
  h->steps_done = s0 + nsteps;
  if (hipGetLastError() != hipSuccess) return HGKS_E_DEVICE;
  return hip_status(hipStreamSynchronize(st));
}

int hgks_operator(hgks_handle* h, const double* q_in, double dt, double* L, double* dL) {
  if (!h || !q_in || !L || !dL) return HGKS_E_INVALID_ARG;
  if (h->p.mode != HGKS_MODE_SMOOTH) {
    // the full flux is integrated over the step: it needs dt
    if (!(dt > 0.0)) return HGKS_E_INVALID_ARG;
    launch_set_dt(h->ctrl, dt, h->stream);
  }
  all_fluxes(h, q_in, false, &h->ctrl->zero);
  if (f32(h))
    launch_operator(h->geo, fl_dir<float>(h, 0), L, dL, h->stream);
  else
    launch_operator(h->geo, fl_dir<double>(h, 0), L, dL, h->stream);
  return hip_status(hipGetLastError());
}

int hgks_face_flux(hgks_handle* h, int32_t dir, const double* q_in, double dt, double* F, double* dF) {
  if (!h || !q_in || !F || !dF || dir < 0 || dir > 2) return HGKS_E_INVALID_ARG;
  const Geo& g = h->geo;
  if (h->p.mode != HGKS_MODE_SMOOTH) {
    if (!(dt > 0.0)) return HGKS_E_INVALID_ARG;
    launch_set_dt(h->ctrl, dt, h->stream);
  }
  if (f32(h)) {
    mode_flux(h, dir, false, q_in, fl_dir<float>(h, dir), &h->ctrl->zero);
    launch_export_flux(g, dir, fl_dir<float>(h, dir), F, dF, h->stream);
  } else {
    mode_flux(h, dir, false, q_in, fl_dir<double>(h, dir), &h->ctrl->zero);
    launch_export_flux(g, dir, fl_dir<double>(h, dir), F, dF, h->stream);
  }
  return hip_status(hipGetLastError());
}

int hgks_wall_flux(hgks_handle* h, const double* q_in, double* F, double* dF) {
  if (!h || !q_in || !F || !dF) return HGKS_E_INVALID_ARG;
  if (!h->geo.wall_y) return HGKS_E_UNSUPPORTED;
  const Geo& g = h->geo;
  if (f32(h)) {
    launch_flux_fused(g, 1, false, q_in, fl_dir<float>(h, 1), &h->ctrl->zero, h->stream);
    launch_export_wall_flux(g, fl_dir<float>(h, 1), F, dF, h->stream);
  } else {
    launch_flux_fused(g, 1, false, q_in, fl_dir<double>(h, 1), &h->ctrl->zero, h->stream);
    launch_export_wall_flux(g, fl_dir<double>(h, 1), F, dF, h->stream);
  }
  return hip_status(hipGetLastError());
}

int hgks_step_vjp(hgks_handle* h, const double* q_n, double dt, const double* lam_np1, double* lam_n) {
  if (!h || !q_n || !lam_np1 || !lam_n || !(dt > 0.0)) return HGKS_E_INVALID_ARG;
  if (lam_n == lam_np1 || lam_n == q_n) return HGKS_E_INVALID_ARG;
  if (h->geo.wall_y || h->geo.stretch_y || h->geo.fx != 0.0 || h->mflux) return HGKS_E_UNSUPPORTED;
  // smooth mode: constant viscosity, FP64 or the FP32-flux form; mode Z: FP64
  if (h->p.mode == HGKS_MODE_SMOOTH && h->p.mu_exp != 0.0) return HGKS_E_UNSUPPORTED;
  if (h->p.mode == HGKS_MODE_WENOZ_CHAR) return HGKS_E_UNSUPPORTED;
  if (h->p.mode == HGKS_MODE_WENOZ && f32(h)) return HGKS_E_UNSUPPORTED;
  const Geo& g = h->geo;
  hipStream_t st = h->stream;
  const long long n5 = 5 * g.N;
  // forward stage 1 with the frozen time step: Q* into the workspace
  launch_set_dt(h->ctrl, dt, st);
  all_fluxes(h, q_n, false, &h->ctrl->zero);
  stage1(h, q_n, h->qs, -1);
  // lambda* = (ddL/dQ)^T(Q*) (dt^2/3 lambda); the operator VJP's scratch starts
  // from zeros (it leaves it cleared)
  if (h->p.mode == HGKS_MODE_SMOOTH) launch_fill(vjp_scratch(h), 0.0, 10 * g.N, st);
  launch_fill(h->lam_star, 0.0, n5, st);
  operator_vjp(h, h->qs, lam_np1, nullptr, 0.0, 0.0, dt * dt / 3.0, 0.0, h->lam_star);
  // lambda_n = lambda + lambda* + (dL/dQ)^T(Q^n) (dt lambda + dt/2 lambda*)
  //                              + (ddL/dQ)^T(Q^n) (dt^2/6 lambda + dt^2/8 lambda*)
  launch_axpby(1.0, lam_np1, 1.0, h->lam_star, lam_n, n5, st);
  operator_vjp(h, q_n, lam_np1, h->lam_star, dt, 0.5 * dt, dt * dt / 6.0, dt * dt / 8.0, lam_n);
  return hip_status(hipGetLastError());
}

int hgks_diagnostics(hgks_handle* h, double* out) {
  if (!h || !out) return HGKS_E_INVALID_ARG;
  launch_diagnostics(h->geo, h->q, h->diag_part, h->diag_out, h->stream);
  if (hipGetLastError() != hipSuccess) return HGKS_E_DEVICE;
  if (hipMemcpyAsync(out, h->diag_out, sizeof(double) * HGKS_NDIAG, hipMemcpyDeviceToHost, h->stream) != hipSuccess)
    return HGKS_E_DEVICE;
  return hip_status(hipStreamSynchronize(h->stream));
}

static_assert(HGKS_PDF_MAX_BINS == kPdfMaxBins, "one bin limit");

int hgks_dilatation_pdf(hgks_handle* h, int32_t nbins, double lo, double hi, int64_t* counts, double* theta_rms) {
  if (!h || !counts || !theta_rms || nbins < 1 || nbins > HGKS_PDF_MAX_BINS) return HGKS_E_INVALID_ARG;
  if (!std::isfinite(lo) || !std::isfinite(hi) || !(lo < hi) || !std::isfinite(hi - lo)) return HGKS_E_INVALID_ARG;
  if (h->geo.stretch_y) return HGKS_E_UNSUPPORTED;
  launch_dilatation_pdf(h->geo, h->q, h->diag_part, nbins, lo, hi, h->stream);
  if (hipGetLastError() != hipSuccess) return HGKS_E_DEVICE;
  if (hipMemcpyAsync(theta_rms, h->diag_part + dilatation_pdf_rms_offset(), sizeof(double), hipMemcpyDeviceToHost,
                     h->stream) != hipSuccess)
    return HGKS_E_DEVICE;
  if (hipMemcpyAsync(counts, h->diag_part + dilatation_pdf_counts_offset(), sizeof(int64_t) * size_t(nbins + 2),
                     hipMemcpyDeviceToHost, h->stream) != hipSuccess)
    return HGKS_E_DEVICE;
  return hip_status(hipStreamSynchronize(h->stream));
}

int hgks_dilatation_slice(hgks_handle* h, int32_t axis, int32_t index, double* out, double* theta_rms) {
  if (!h || !out || !theta_rms || axis < 0 || axis > 2) return HGKS_E_INVALID_ARG;
  if (index < 0 || index >= h->geo.n[axis]) return HGKS_E_INVALID_ARG;
  if (h->geo.stretch_y) return HGKS_E_UNSUPPORTED;
  const int fa = axis == 0 ? 1 : 0, sa = axis == 2 ? 1 : 2;
  const size_t cells = size_t(h->geo.n[fa]) * size_t(h->geo.n[sa]);  // < N / 6, inside the face-flux arrays
  double* scratch = reinterpret_cast<double*>(h->fl);
  launch_dilatation_slice(h->geo, h->q, h->diag_part, axis, index, scratch, h->stream);
  if (hipGetLastError() != hipSuccess) return HGKS_E_DEVICE;
  if (hipMemcpyAsync(theta_rms, h->diag_part + dilatation_pdf_rms_offset(), sizeof(double), hipMemcpyDeviceToHost,
                     h->stream) != hipSuccess)
    return HGKS_E_DEVICE;
  if (hipMemcpyAsync(out, scratch, sizeof(double) * cells, hipMemcpyDeviceToHost, h->stream) != hipSuccess)
    return HGKS_E_DEVICE;
  return hip_status(hipStreamSynchronize(h->stream));
}

static_assert(HGKS_NPROFILE == kNProfile, "one profile width");

int hgks_plane_profiles(hgks_handle* h, double* out) {
  if (!h || !out) return HGKS_E_INVALID_ARG;
  // ny rows of kNProfile doubles; the face-flux arrays hold at least 15 N >= 540 ny doubles
  double* scratch = reinterpret_cast<double*>(h->fl);
  launch_plane_profiles(h->geo, h->q, scratch, h->stream);
  if (hipGetLastError() != hipSuccess) return HGKS_E_DEVICE;
  if (hipMemcpyAsync(out, scratch, sizeof(double) * size_t(kNProfile) * size_t(h->geo.n[1]), hipMemcpyDeviceToHost,
                     h->stream) != hipSuccess)
    return HGKS_E_DEVICE;
  return hip_status(hipStreamSynchronize(h->stream));
}

int hgks_profile_enable(hgks_handle* h, int enable) {
  if (!h) return HGKS_E_INVALID_ARG;
  if (!enable) {
    if (hipStreamSynchronize(h->stream) != hipSuccess) return HGKS_E_DEVICE;
    for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
    h->events.clear();
    h->pending_class.clear();
  }
  h->profiling = enable != 0;
  return HGKS_OK;
}

int hgks_profile_read(hgks_handle* h, double* ms, int64_t* counts, int n) {
  if (!h || !ms || !counts || n < 0 || n > HGKS_KCLASS_COUNT) return HGKS_E_INVALID_ARG;
  if (hipStreamSynchronize(h->stream) != hipSuccess) return HGKS_E_DEVICE;
  prof_collect(h);
  for (int k = 0; k < n; ++k) {
    ms[k] = h->prof_ms[k];
    counts[k] = h->prof_count[k];
  }
  for (int k = 0; k < HGKS_KCLASS_COUNT; ++k) { h->prof_ms[k] = 0.0; h->prof_count[k] = 0; }
  return HGKS_OK;
}

int hgks_failed_step(const hgks_handle* h) { return h ? h->failed_step : -1; }

void hgks_destroy(hgks_handle* h) {
  if (!h) return;
  if (!h->events.empty()) {
    (void)hipStreamSynchronize(h->stream);
    for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
  }
  delete h;
}

const char* hgks_strerror(int status) {
  switch (status) {
    case HGKS_OK: return "ok";
    case HGKS_E_INVALID_ARG: return "invalid argument";
    case HGKS_E_DEVICE: return "HIP runtime error";
    case HGKS_E_NONPHYSICAL: return "non-physical state (rho <= 0, p <= 0 or non-finite)";
    case HGKS_E_UNSUPPORTED: return "unsupported parameter combination";
    case HGKS_E_WORKSPACE: return "workspace missing, too small or misaligned";
    default: return "unknown status";
  }
}

}  // extern "C"
