// gpe_api.hip -- host side of libgpe: parameter validation and stability
// estimates, workspace layout, the per-step launch sequence, HIP-graph
// replay, diagnostics and field transfer.  Implements include/gpe.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "gpe.h"
#include "gpe_device.hpp"
#include "gpe_host.hpp"
#include "gpe_misc.hpp"

namespace {

using gpe::ChArgs;
using gpe::Consts;
using gpe::FlowArgs;
using gpe::Grid;
using namespace gpe_host;

int dim_of(const gpe_params* p) { return p->geometry == GPE_GEOM_3D ? 3 : 2; }

// Which workspace buffers a parameter set needs.
void needed(const gpe_params* p, bool need[B_COUNT]) {
  const int dim = dim_of(p);
  for (int b = 0; b < B_COUNT; ++b) need[b] = true;
  if (dim == 2) {
    need[B_Q0 + 2] = need[B_Q1 + 2] = need[B_Q2 + 2] = false;  // no Y velocity
    need[B_US + 1] = false;
    need[B_PHB] = false;                                       // RK2 only
  }
}

size_t scratch_bytes() { return (size_t)(gpe::kDiagBlocks * 8 + 8) * sizeof(double); }

int validate(const gpe_params* p) {
  if (!p) return GPE_EINVAL;
  if (p->geometry < 0 || p->geometry > 2) return GPE_EINVAL;
  if (p->precision != GPE_FP64 && p->precision != GPE_FP32) return GPE_EINVAL;
  const int dim = dim_of(p);
  for (int a = 0; a < 3; ++a) {
    if (a < dim) {
      if (p->n[a] < 3) return GPE_EINVAL;
    } else if (p->n[a] != 1) {
      return GPE_EINVAL;
    }
  }
  const double ncell = (double)p->n[0] * p->n[1] * p->n[2];
  if (ncell > 4.0e9) return GPE_EINVAL;
  // one Z plane (X x Y in the internal axis order, rows padded to the row
  // pitch) must stay below 2^32 bytes
  const double esize = p->precision == GPE_FP64 ? 8.0 : 4.0;
  const double pitch = (double)row_pitch(p);
  const double plane = dim == 3 ? pitch * p->n[1] : pitch;
  if (plane * esize >= 4294967296.0) return GPE_EINVAL;
  for (int a = 0; a < dim; ++a) {
    const int lo = p->bc[2 * a], hi = p->bc[2 * a + 1];
    if (lo < 0 || lo > 2 || hi < 0 || hi > 2) return GPE_EINVAL;
    if ((lo == GPE_BC_PERIODIC) != (hi == GPE_BC_PERIODIC)) return GPE_EINVAL;
  }
  if (dim == 2 && p->lattice != GPE_D2Q9) return GPE_EINVAL;
  if (dim == 3 && p->lattice != GPE_D3Q15 && p->lattice != GPE_D3Q19 && p->lattice != GPE_D3Q27)
    return GPE_EINVAL;
  if (p->geometry == GPE_GEOM_AXISYM) {
    if (p->bc[2] != GPE_BC_SYMMETRY) return GPE_EINVAL;  // the axis
    if (p->g[1] != 0.0) return GPE_EINVAL;               // body force along the axis only
  }
  if (!(p->dt > 0) || !(p->cs2 > 0)) return GPE_EINVAL;
  if (!(p->rho_l > 0) || !(p->rho_g > 0)) return GPE_EINVAL;
  if (!(p->eta_l >= 0) || !(p->eta_g >= 0)) return GPE_EINVAL;
  if (!(p->sigma >= 0) || !(p->mobility >= 0) || !(p->width > 0)) return GPE_EINVAL;
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(p->g[a])) return GPE_EINVAL;
  if (!std::isfinite(p->rho_ref)) return GPE_EINVAL;
  if (p->ch_transport != GPE_CH_CONSERVATIVE && p->ch_transport != GPE_CH_ADVECTIVE) return GPE_EINVAL;
  if (p->scheme < 0 || p->scheme > (GPE_SCHEME_NO_PAVG | GPE_SCHEME_NO_BULK)) return GPE_EINVAL;
  if (p->scheme != GPE_SCHEME_PAPER && dim != 3) return GPE_EINVAL;
  if (p->init_kind < 0 || p->init_kind > 4) return GPE_EINVAL;
  if (p->zchunk < 0) return GPE_EINVAL;
  if (p->init_kind == GPE_INIT_ELLIPSE && (!(p->init_radius > 0) || !(std::fabs(p->init_amp) < 1.0)))
    return GPE_EINVAL;
  return GPE_OK;
}

void lattice_weights(int lattice, double w[4]) {
  switch (lattice) {
    case GPE_D2Q9: w[0] = 4.0 / 9; w[1] = 1.0 / 9; w[2] = 1.0 / 36; w[3] = 0; break;
    case GPE_D3Q15: w[0] = 2.0 / 9; w[1] = 1.0 / 9; w[2] = 0; w[3] = 1.0 / 72; break;
    case GPE_D3Q19: w[0] = 1.0 / 3; w[1] = 1.0 / 18; w[2] = 1.0 / 36; w[3] = 0; break;
    default: w[0] = 8.0 / 27; w[1] = 2.0 / 27; w[2] = 1.0 / 54; w[3] = 1.0 / 216; break;
  }
}

// Largest eigenvalue of minus the isotropic Laplacian symbol,
// 6 sum_i w_i (1 - cos(k . e_i)), scanned over the Brillouin zone.
double iso_lap_max(int lattice, int dim) {
  double w[4];
  lattice_weights(lattice, w);
  const int N = 24;
  double best = 0;
  for (int a = 0; a <= N; ++a)
    for (int b = 0; b <= N; ++b)
      for (int c = 0; c <= (dim == 3 ? N : 0); ++c) {
        const double k[3] = {M_PI * a / N, M_PI * b / N, M_PI * c / N};
        double s = 0;
        for (int ez = -1; ez <= 1; ++ez) {
          if (dim == 2 && ez != 0) continue;
          for (int ey = -1; ey <= 1; ++ey)
            for (int ex = -1; ex <= 1; ++ex) {
              const int nnz = (ex != 0) + (ey != 0) + (ez != 0);
              if (nnz == 0) continue;
              s += w[nnz] * (1 - std::cos(k[0] * ex + k[1] * ey + k[2] * ez));
            }
        }
        best = std::fmax(best, 6 * s);
      }
  return best;
}

// Linear stability estimates (returns the largest ratio to its limit).
double stability_ratio(const gpe_params* p) {
  const int d = dim_of(p);
  const double cs = std::sqrt(p->cs2);
  // acoustic: |lambda dt| = 2 c_s dt with the averaged pressure gradient;
  // TVD-RK3 is stable on the imaginary axis up to sqrt(3)
  double r = 2.0 * cs * p->dt / std::sqrt(3.0);
  const double nu_max = std::fmax(p->eta_l / p->rho_l, p->eta_g / p->rho_g);
  // compressive viscous mode 3 nu |k|^2 <= 3 nu 4 d; RK3 real-axis limit 2.5127
  r = std::fmax(r, 3.0 * nu_max * p->dt * 4.0 * d / 2.5127);
  // CH linearised about phi = +-1: M lam (8a + kappa lam), RK2 limit 2, RK4 2.785
  const double a = 3.0 / (4.0 * p->width), kappa = 3.0 * p->width / 8.0;
  const double lam = iso_lap_max(p->lattice, d);
  const double ch = p->mobility * p->dt * lam * (8.0 * a + kappa * lam);
  r = std::fmax(r, ch / (d == 3 ? 2.785 : 2.0));
  return r;
}

template <typename T>
Consts<T> make_consts(const gpe_params* p, int dim) {
  Consts<T> c;
  double w[4];
  lattice_weights(p->lattice, w);
  c.dt = T(p->dt);
  c.cs2 = T(p->cs2);
  c.rho_l = T(p->rho_l);
  c.rho_g = T(p->rho_g);
  c.eta_l = T(p->eta_l);
  c.eta_g = T(p->eta_g);
  c.sigma = T(p->sigma);
  c.mob = T(p->mobility);
  c.a4 = T(4.0 * 3.0 / (4.0 * p->width));
  c.kappa6 = T(6.0 * 3.0 * p->width / 8.0);
  c.rho_ref = T(p->rho_ref);
  if (dim == 3) {
    c.g[0] = T(p->g[0]); c.g[1] = T(p->g[1]); c.g[2] = T(p->g[2]);
  } else {
    c.g[0] = T(p->g[0]); c.g[1] = T(0); c.g[2] = T(p->g[1]);
  }
  c.w1 = T(w[1]);
  c.w2 = T(w[2]);
  c.w3 = T(w[3]);
  c.rho_a = T(0.5 * (p->rho_l + p->rho_g));
  c.rho_hb = T(0.25 * (p->rho_l - p->rho_g));
  c.eta_a = T(0.5 * (p->eta_l + p->eta_g));
  c.eta_b = T(0.5 * (p->eta_l - p->eta_g));
  c.hsig = T(-0.5 * p->sigma);
  return c;
}

// ---- kernel sequence of one time step ----------------------------------
// Chained timing events: one before the first kernel of a step and one after
// every kernel, so kernel q of a step lasts from event q to event q + 1.
// Only the boundaries of the kernels selected by mask get an event.
struct KernelTimer {
  hipEvent_t* ev = nullptr;  // this step's events
  int n = 0;
  uint32_t mask = ~0u;
  bool wants(int q) const { return ((mask >> q) & 1u) || (q > 0 && ((mask >> (q - 1)) & 1u)); }
};

// Longest Z chunk per work-group (planes): see choose_zchunk.
int zchunk_max(size_t esize) { return esize == 8 ? 128 : 64; }

// Rows per work-group of a 2-D grid.  A 2-D work-group is one wave on a
// 64-column strip, and a single 2-D grid gives few of them: a launch then
// lasts about as long as one work-group takes to stage its first rows and
// march its own, each row waiting on the loads issued one row earlier, times
// the rounds of work-groups the device needs.  The chunk minimises
// rounds x (rows + 3 staged warm-up rows) over 1 .. zmax rows; smaller
// chunks win ties.  On MI355X this halves the step of grids up to 256 x 256
// against chunks of 8 rows or more, and it picks the measured best chunk on
// 64^2, 256^2, 96 x 32 and 256 x 1024.
int rows_2d(const int n[3], int tx, int bpc, int ncu, int zmax) {
  const long tiles = (n[0] + tx - 1) / tx;
  const long slots = (long)ncu * bpc;
  int best = 1;
  long best_t = -1;
  for (int zc = 1; zc <= std::min(n[2], zmax); ++zc) {
    const long w = tiles * ((n[2] + zc - 1) / zc);
    const long t = (w + slots - 1) / slots * (zc + 3);
    if (best_t < 0 || t < best_t) {
      best_t = t;
      best = zc;
    }
  }
  return best;
}

int flow_zchunk(const gpe_state* s, size_t esize) {
  if (s->P.zchunk > 0) return std::min(s->P.zchunk, s->grid.n[2]);
  const int zmax = zchunk_max(esize);
  if (s->dim == 3)
    return esize == 8 ? gpe::choose_zchunk(s->grid.n, gpe::FlowTile<3, double>::TX, gpe::FlowTile<3, double>::TY,
                                           gpe::FlowTile<3, double>::BPC, s->ncu, zmax)
                      : gpe::choose_zchunk(s->grid.n, gpe::FlowTile<3, float>::TX, gpe::FlowTile<3, float>::TY,
                                           gpe::FlowTile<3, float>::BPC, s->ncu, zmax);
  return rows_2d(s->grid.n, gpe::FlowTile<2, float>::TX, gpe::FlowTile<2, float>::BPC, s->ncu, zmax);
}

int ch_zchunk(const gpe_state* s, size_t esize) {
  if (s->P.zchunk > 0) return std::min(s->P.zchunk, s->grid.n[2]);
  const int zmax = zchunk_max(esize);
  if (s->dim == 3)
    return esize == 8 ? gpe::choose_zchunk(s->grid.n, gpe::ChTile<3, double>::TX, gpe::ChTile<3, double>::TY,
                                           gpe::ChTile<3, double>::BPC, s->ncu, zmax)
                      : gpe::choose_zchunk(s->grid.n, gpe::ChTile<3, float>::TX, gpe::ChTile<3, float>::TY,
                                           gpe::ChTile<3, float>::BPC, s->ncu, zmax);
  return rows_2d(s->grid.n, gpe::ChTile<2, float>::TX, gpe::ChTile<2, float>::BPC, s->ncu, zmax);
}

template <typename T>
hipError_t enqueue_step_t(gpe_state* s, KernelTimer* kt) {
  const int geom = s->P.geometry;
  hipError_t e = hipSuccess;
  auto mark = [&]() {
    if (!kt) return;
    if (kt->wants(kt->n)) (void)hipEventRecord(kt->ev[kt->n], s->stream);
    ++kt->n;
  };
  mark();
  const int zf = flow_zchunk(s, sizeof(T));
  for (int st = 1; st <= 3; ++st) {
    e = gpe::launch_flow<T>(flow_args<T>(s, st, zf), geom, st, s->P.scheme, s->stream);
    mark();
    if (e != hipSuccess) return e;
  }
  ChArgs<T> h[4];
  int stage[4];
  const int nch = ch_args<T>(s, ch_zchunk(s, sizeof(T)), h, stage);
  for (int q = 0; q < nch; ++q) {
    e = gpe::launch_ch<T>(h[q], geom, stage[q], s->stream);
    mark();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t enqueue_step(gpe_state* s, KernelTimer* kt = nullptr) {
  return s->P.precision == GPE_FP64 ? enqueue_step_t<double>(s, kt) : enqueue_step_t<float>(s, kt);
}

template <typename T>
hipError_t enqueue_diag_t(gpe_state* s) {
  gpe::DiagArgs<T> d;
  d.g = s->grid;
  d.axisym = s->axi ? 1 : 0;
  d.rho_l = s->P.rho_l;
  d.rho_g = s->P.rho_g;
  d.phi = buf<T>(s, B_PHI);
  for (int q = 0; q < 4; ++q) d.q[q] = buf<T>(s, B_Q0 + q);
  d.partial = buf<double>(s, B_SCR);
  d.result = d.partial + gpe::kDiagBlocks * 8;
  return gpe::launch_diag<T>(d, s->stream);
}

int run_diag(gpe_state* s, double out[8]) {
  hipError_t e = s->P.precision == GPE_FP64 ? enqueue_diag_t<double>(s) : enqueue_diag_t<float>(s);
  if (e != hipSuccess) return GPE_EHIP;
  const double* res = buf<double>(s, B_SCR) + gpe::kDiagBlocks * 8;
  if (hipMemcpyAsync(out, res, 8 * sizeof(double), hipMemcpyDeviceToHost, s->stream) != hipSuccess)
    return GPE_EHIP;
  if (hipStreamSynchronize(s->stream) != hipSuccess) return GPE_EHIP;
  return GPE_OK;
}

// External field id -> internal buffer.
int field_buf(const gpe_state* s, int field) {
  switch (field) {
    case GPE_FIELD_P: return B_Q0 + 0;
    case GPE_FIELD_U: return B_Q0 + 1;
    case GPE_FIELD_V: return s->dim == 3 ? B_Q0 + 2 : B_Q0 + 3;
    case GPE_FIELD_W: return s->dim == 3 ? B_Q0 + 3 : -1;
    case GPE_FIELD_PHI: return B_PHI;
  }
  return -1;
}

// Host array of the cells in the a0 order (rows of nx) <-> the padded rows
// of a field buffer.
hipError_t copy_rows(gpe_state* s, void* dev, void* host, size_t esize, int dir) {
  const size_t nx = (size_t)s->grid.n[0], rows = s->ncell / nx, pitch = (size_t)s->grid.pitch;
  if (pitch == nx)
    return dir == GPE_H2D ? hipMemcpyAsync(dev, host, s->ncell * esize, hipMemcpyHostToDevice, s->stream)
                          : hipMemcpyAsync(host, dev, s->ncell * esize, hipMemcpyDeviceToHost, s->stream);
  return dir == GPE_H2D
             ? hipMemcpy2DAsync(dev, pitch * esize, host, nx * esize, nx * esize, rows, hipMemcpyHostToDevice, s->stream)
             : hipMemcpy2DAsync(host, nx * esize, dev, pitch * esize, nx * esize, rows, hipMemcpyDeviceToHost,
                                s->stream);
}

template <typename T>
int copy_t(gpe_state* s, int b, int dir, double* host) {
  T* dev = buf<T>(s, b);
  const size_t n = s->ncell;
  if (sizeof(T) == sizeof(double)) {
    if (copy_rows(s, dev, host, sizeof(T), dir) != hipSuccess || hipStreamSynchronize(s->stream) != hipSuccess)
      return GPE_EHIP;
    return GPE_OK;
  }
  std::vector<T> tmp(n);
  if (dir == GPE_H2D) {
    for (size_t c = 0; c < n; ++c) tmp[c] = T(host[c]);
    if (copy_rows(s, dev, tmp.data(), sizeof(T), dir) != hipSuccess || hipStreamSynchronize(s->stream) != hipSuccess)
      return GPE_EHIP;
  } else {
    if (copy_rows(s, dev, tmp.data(), sizeof(T), dir) != hipSuccess || hipStreamSynchronize(s->stream) != hipSuccess)
      return GPE_EHIP;
    for (size_t c = 0; c < n; ++c) host[c] = (double)tmp[c];
  }
  return GPE_OK;
}

template <typename T>
int init_fields_t(gpe_state* s, const double* h_phi0, const double* h_p0) {
  const gpe_params& P = s->P;
  gpe::InitArgs<T> a;
  for (int q = 0; q < 3; ++q) a.n[q] = s->grid.n[q];
  a.pitch = s->grid.pitch;
  a.kind = h_phi0 ? 0 : P.init_kind;
  a.has_y = s->dim == 3;
  if (s->dim == 3) {
    for (int q = 0; q < 3; ++q) a.center[q] = P.init_center[q];
  } else {
    a.center[0] = P.init_center[0];
    a.center[1] = 0.0;
    a.center[2] = P.init_center[1];
  }
  a.radius = P.init_radius;
  a.width = P.init_width > 0 ? P.init_width : P.width;
  a.amp = P.init_amp;
  a.phi = buf<T>(s, B_PHI);
  for (int q = 0; q < 4; ++q) a.q[q] = buf<T>(s, B_Q0 + q);
  if (gpe::launch_init<T>(a, s->stream) != hipSuccess) return GPE_EHIP;
  if (h_phi0) {
    int r = copy_t<T>(s, B_PHI, GPE_H2D, const_cast<double*>(h_phi0));
    if (r) return r;
  }
  if (h_p0) {
    int r = copy_t<T>(s, B_Q0, GPE_H2D, const_cast<double*>(h_p0));
    if (r) return r;
  }
  return GPE_OK;
}

}  // namespace

namespace gpe_host {

template <typename T>
FlowArgs<T> flow_args(const gpe_state* s, int st, int zchunk) {
  FlowArgs<T> f;
  f.g = s->grid;
  f.g.zchunk = zchunk;
  f.c = make_consts<T>(&s->P, s->dim);
  f.phi = buf<T>(s, B_PHI);
  for (int a = 0; a < 3; ++a) f.usum[a] = buf<T>(s, B_US + a);
  // mu of the frozen phi lives in CH stage buffer A during the flow step (the
  // CH sub-step's first stage overwrites that buffer before anything reads it)
  f.mu = buf<T>(s, B_PHA);
  const int src = st == 1 ? B_Q0 : (st == 2 ? B_Q1 : B_Q2);
  const int dst = st == 1 ? B_Q1 : (st == 2 ? B_Q2 : B_Q0);
  for (int q = 0; q < 4; ++q) {
    f.src[q] = buf<T>(s, src + q);
    f.qn[q] = buf<T>(s, B_Q0 + q);
    f.dst[q] = buf<T>(s, dst + q);
  }
  return f;
}

template <typename T>
int ch_args(const gpe_state* s, int zchunk, ChArgs<T> a[4], int stage[4]) {
  ChArgs<T> h;
  h.g = s->grid;
  h.g.zchunk = zchunk;
  h.c = make_consts<T>(&s->P, s->dim);
  h.adv = s->P.ch_transport == GPE_CH_ADVECTIVE ? 1 : 0;
  for (int q = 0; q < 3; ++q) h.usum[q] = buf<T>(s, B_US + q);
  T* phi = buf<T>(s, B_PHI);
  T* pa = buf<T>(s, B_PHA);
  T* pb = buf<T>(s, B_PHB);
  h.phis = phi;
  h.acc = buf<T>(s, B_ACC);
  struct Stg { int stage; T* in; T* out; };
  const Stg rk2[2] = {{gpe::CH_RK2_1, phi, pa}, {gpe::CH_RK2_2, pa, phi}};
  const Stg rk4[4] = {{gpe::CH_RK4_1, phi, pa}, {gpe::CH_RK4_2, pa, pb}, {gpe::CH_RK4_3, pb, pa},
                      {gpe::CH_RK4_4, pa, phi}};
  const int n = s->dim == 2 ? 2 : 4;
  for (int q = 0; q < n; ++q) {
    const Stg& t = s->dim == 2 ? rk2[q] : rk4[q];
    a[q] = h;
    a[q].phi_in = t.in;
    a[q].out = t.out;
    stage[q] = t.stage;
  }
  return n;
}

template FlowArgs<float> flow_args<float>(const gpe_state*, int, int);
template FlowArgs<double> flow_args<double>(const gpe_state*, int, int);
template int ch_args<float>(const gpe_state*, int, ChArgs<float>*, int*);
template int ch_args<double>(const gpe_state*, int, ChArgs<double>*, int*);

}  // namespace gpe_host

extern "C" {

int gpe_params_from_dimensionless(const gpe_problem* in, gpe_params* out) {
  if (!in || !out) return GPE_EINVAL;
  const double N_L = in->N_L;
  if (!(N_L > 0) || !(in->r_rho > 0) || !(in->r_eta > 0) || !(in->Cn > 0) || !(in->Pe >= 0))
    return GPE_EINVAL;
  std::memset(out, 0, sizeof(*out));
  out->geometry = in->geometry;
  out->precision = in->precision;
  for (int a = 0; a < 3; ++a) out->n[a] = in->n[a];
  for (int a = 0; a < 6; ++a) out->bc[a] = in->bc[a];
  out->lattice = in->lattice;
  out->ch_transport = in->ch_transport;
  out->scheme = in->scheme;
  // dx = L_c / N_L = 1 and dt = 1; c_s = dx / (sqrt(3) dt)
  out->dt = 1.0;
  out->cs2 = 1.0 / 3.0;
  double Uc;
  if (in->time_scale == GPE_TIME_NT) {
    if (!(in->N_t > 0)) return GPE_EINVAL;
    Uc = N_L / in->N_t;
  } else if (in->time_scale == GPE_TIME_MA) {
    if (!(in->Ma > 0)) return GPE_EINVAL;
    Uc = in->Ma * std::sqrt(out->cs2);
  } else {
    return GPE_EINVAL;
  }
  const double rho_l = 1.0, rho_g = rho_l / in->r_rho, drho = rho_l - rho_g;
  out->rho_l = rho_l;
  out->rho_g = rho_g;
  const double Lg = N_L * (in->L_g_factor > 0 ? in->L_g_factor : 1.0);
  // direction and, for G and Fr, magnitude of the body force
  const double gn = std::sqrt(in->G[0] * in->G[0] + in->G[1] * in->G[1] + in->G[2] * in->G[2]);
  double gmag = -1.0;  // < 0: not yet known
  if (in->gravity == GPE_GRAV_G) {
    gmag = gn * Uc * Uc / N_L;
  } else if (in->gravity == GPE_GRAV_FR) {
    if (!(in->Fr > 0) || !(gn > 0)) return GPE_EINVAL;
    gmag = Uc * Uc / (in->Fr * in->Fr * N_L);
  } else if (in->gravity == GPE_GRAV_EO) {
    if (!(in->Eo > 0) || !(gn > 0) || !(drho > 0) || in->st_group == GPE_ST_EO) return GPE_EINVAL;
  } else {
    return GPE_EINVAL;
  }
  // surface tension when it does not depend on eta_L
  double sigma = -1.0;
  switch (in->st_group) {
    case GPE_ST_NONE: sigma = 0.0; break;
    case GPE_ST_WE:
      if (!(in->We > 0)) return GPE_EINVAL;
      sigma = rho_l * Uc * Uc * N_L / in->We;
      break;
    case GPE_ST_EO:
      if (!(in->Eo > 0) || !(gmag > 0) || !(drho > 0)) return GPE_EINVAL;
      sigma = gmag * drho * Lg * Lg / in->Eo;
      break;
    case GPE_ST_SIGMA:
      if (!(in->sigma >= 0)) return GPE_EINVAL;
      sigma = in->sigma;
      break;
    case GPE_ST_CAPILLARY: break;  // sigma = U_c eta_L below
    default: return GPE_EINVAL;
  }
  const bool capillary = in->st_group == GPE_ST_CAPILLARY;
  double eta_l;
  switch (in->visc_group) {
    case GPE_VISC_RE:
      if (!(in->Re > 0)) return GPE_EINVAL;
      eta_l = rho_l * Uc * N_L / in->Re;
      break;
    case GPE_VISC_OH:
      if (!(in->Oh > 0)) return GPE_EINVAL;
      // Oh^2 = eta_L^2 / (rho_L sigma L_g); with sigma = U_c eta_L it is linear in eta_L
      eta_l = capillary ? in->Oh * in->Oh * rho_l * Uc * Lg : in->Oh * std::sqrt(rho_l * sigma * Lg);
      if (!capillary && !(sigma > 0)) return GPE_EINVAL;
      break;
    case GPE_VISC_MO:
      if (!(in->Mo > 0) || !(gmag > 0) || !(drho > 0)) return GPE_EINVAL;
      if (capillary) {
        eta_l = in->Mo * rho_l * rho_l * Uc * Uc * Uc / (gmag * drho);
      } else {
        if (!(sigma > 0)) return GPE_EINVAL;
        eta_l = std::pow(in->Mo * rho_l * rho_l * sigma * sigma * sigma / (gmag * drho), 0.25);
      }
      break;
    case GPE_VISC_CAPILLARY:
      if (capillary || !(sigma > 0)) return GPE_EINVAL;
      eta_l = sigma / Uc;
      break;
    default: return GPE_EINVAL;
  }
  if (capillary) sigma = Uc * eta_l;
  if (in->gravity == GPE_GRAV_EO) gmag = in->Eo * sigma / (drho * Lg * Lg);
  out->eta_l = eta_l;
  out->eta_g = eta_l / in->r_eta;
  out->sigma = sigma;
  out->mobility = in->Pe > 0 ? Uc * N_L * N_L / in->Pe : 0.0;  // sigma_ref = 1
  out->width = in->Cn * N_L;
  for (int a = 0; a < 3; ++a) out->g[a] = gn > 0 ? gmag * in->G[a] / gn : 0.0;
  switch (in->rho_ref_kind) {
    case GPE_RHO_REF_ZERO: out->rho_ref = 0.0; break;
    case GPE_RHO_REF_LIQUID: out->rho_ref = rho_l; break;
    case GPE_RHO_REF_GAS: out->rho_ref = rho_g; break;
    case GPE_RHO_REF_VALUE: out->rho_ref = in->rho_ref_value * rho_l; break;
    default: return GPE_EINVAL;
  }
  return validate(out) == GPE_OK ? GPE_OK : GPE_EINVAL;
}

size_t gpe_workspace_bytes(const gpe_params* p) {
  if (validate(p) != GPE_OK) return 0;
  const size_t esize = p->precision == GPE_FP64 ? 8 : 4;
  const size_t fcell = field_elems(p);
  bool need[B_COUNT];
  needed(p, need);
  size_t total = 0;
  for (int b = 0; b < B_SCR; ++b)
    if (need[b]) total += align_up(fcell * esize);
  total += align_up(scratch_bytes());
  return total;
}

int gpe_init_state(const gpe_params* p, void* d_workspace, size_t bytes, void* hip_stream,
                   const double* h_phi0, const double* h_p0, gpe_state** out) {
  if (!out) return GPE_EINVAL;
  *out = nullptr;
  int v = validate(p);
  if (v) return v;
  if (!p->allow_unstable && stability_ratio(p) > 1.0) return GPE_EUNSTABLE;
  const size_t need_bytes = gpe_workspace_bytes(p);
  if (!d_workspace || bytes < need_bytes || ((uintptr_t)d_workspace % kAlign) != 0)
    return GPE_EWORKSPACE;
  gpe_state* s = new (std::nothrow) gpe_state();
  if (!s) return GPE_EINVAL;
  s->P = *p;
  s->dim = dim_of(p);
  s->axi = p->geometry == GPE_GEOM_AXISYM;
  s->esize = p->precision == GPE_FP64 ? 8 : 4;
  s->ncell = (size_t)p->n[0] * p->n[1] * p->n[2];
  s->fcell = field_elems(p);
  s->stream = (hipStream_t)hip_stream;
  s->ws = (char*)d_workspace;
  s->ws_bytes = bytes;
  s->step = 0;
  s->t = 0.0;
  s->sticky = GPE_OK;
  s->graph_ok = false;
  // internal grid: 3-D as is; 2-D / axisymmetric as (Z = y) x (X = x)
  if (s->dim == 3) {
    for (int a = 0; a < 3; ++a) s->grid.n[a] = p->n[a];
    for (int a = 0; a < 6; ++a) s->grid.bc[a] = p->bc[a];
  } else {
    s->grid.n[0] = p->n[0];
    s->grid.n[1] = 1;
    s->grid.n[2] = p->n[1];
    s->grid.bc[0] = p->bc[0];
    s->grid.bc[1] = p->bc[1];
    s->grid.bc[2] = s->grid.bc[3] = GPE_BC_PERIODIC;
    s->grid.bc[4] = p->bc[2];
    s->grid.bc[5] = p->bc[3];
  }
  s->grid.pitch = (int)row_pitch(p);
  s->grid.zchunk = 1;
  {
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        ncu <= 0)
      ncu = 256;
    s->ncu = ncu;
  }
  bool need[B_COUNT];
  needed(p, need);
  size_t o = 0;
  for (int b = 0; b < B_SCR; ++b) {
    if (need[b]) {
      s->off[b] = o;
      o += align_up(s->fcell * s->esize);
    } else {
      s->off[b] = (size_t)-1;
    }
  }
  s->off[B_SCR] = o;
  // every field buffer starts at zero, the row padding included
  int r = hipMemsetAsync(s->ws, 0, o, s->stream) == hipSuccess ? GPE_OK : GPE_EHIP;
  if (!r)
    r = p->precision == GPE_FP64 ? init_fields_t<double>(s, h_phi0, h_p0) : init_fields_t<float>(s, h_phi0, h_p0);
  double d[8];
  if (!r) r = run_diag(s, d);
  if (r) {
    delete s;
    return r;
  }
  s->mass_abs0 = d[1];
  *out = s;
  return GPE_OK;
}

int gpe_rk3_step(gpe_state* s) {
  if (!s) return GPE_EINVAL;
  if (enqueue_step(s) != hipSuccess) return GPE_EHIP;
  s->step += 1;
  s->t = s->step * s->P.dt;
  return GPE_OK;
}

int gpe_run_n(gpe_state* s, int64_t n) {
  if (!s || n < 0) return GPE_EINVAL;
  if (n == 0) return GPE_OK;
  if (s->stream == nullptr || n < 2) {
    for (int64_t q = 0; q < n; ++q)
      if (enqueue_step(s) != hipSuccess) return GPE_EHIP;
  } else {
    if (!s->graph_ok) {
      hipGraph_t gr;
      if (hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return GPE_EHIP;
      hipError_t e = enqueue_step(s);
      hipError_t e2 = hipStreamEndCapture(s->stream, &gr);
      if (e != hipSuccess || e2 != hipSuccess) return GPE_EHIP;
      e = hipGraphInstantiate(&s->graph, gr, nullptr, nullptr, 0);
      (void)hipGraphDestroy(gr);
      if (e != hipSuccess) return GPE_EHIP;
      s->graph_ok = true;
    }
    for (int64_t q = 0; q < n; ++q)
      if (hipGraphLaunch(s->graph, s->stream) != hipSuccess) return GPE_EHIP;
  }
  s->step += n;
  s->t = s->step * s->P.dt;
  return GPE_OK;
}

int gpe_diagnostics(gpe_state* s, gpe_diag* out) {
  if (!s || !out) return GPE_EINVAL;
  double d[8];
  int r = run_diag(s, d);
  if (r) return r;
  out->step = s->step;
  out->t = s->t;
  out->mass = d[0];
  out->mass_abs0 = s->mass_abs0;
  out->ke = d[2];
  out->max_div = d[3];
  out->phi_min = -d[4];
  out->phi_max = d[5];
  out->umax = d[6];
  out->finite = d[7] == 0.0 ? 1 : 0;
  out->reserved = 0;
  if (!out->finite) s->sticky = GPE_ENONFINITE;
  return s->sticky;
}

int gpe_copy_field(gpe_state* s, int field, int dir, void* host, size_t bytes) {
  if (!s || !host || (dir != GPE_H2D && dir != GPE_D2H)) return GPE_EINVAL;
  const int b = field_buf(s, field);
  if (b < 0) return GPE_EINVAL;
  if (bytes != s->ncell * sizeof(double)) return GPE_EINVAL;
  return s->P.precision == GPE_FP64 ? copy_t<double>(s, b, dir, (double*)host)
                                    : copy_t<float>(s, b, dir, (double*)host);
}

size_t gpe_field_offset(const gpe_state* s, int field) {
  if (!s) return (size_t)-1;
  const int b = field_buf(s, field);
  return b < 0 ? (size_t)-1 : s->off[b];
}

void* gpe_field_pointer(const gpe_state* s, int field) {
  if (!s) return nullptr;
  const int b = field_buf(s, field);
  return b < 0 ? nullptr : (void*)(s->ws + s->off[b]);
}

int64_t gpe_field_pitch(const gpe_state* s) { return s ? (int64_t)s->grid.pitch : GPE_EINVAL; }

int gpe_set_step_time(gpe_state* s, int64_t step, double t) {
  if (!s || step < 0) return GPE_EINVAL;
  s->step = step;
  s->t = t;
  return GPE_OK;
}

int gpe_kernel_times_masked(gpe_state* s, int64_t nsteps, uint32_t mask, int max, const char** names, double* ms,
                            double* bytes) {
  if (!s || nsteps < 1 || max < 1 || !names || !ms || !bytes) return GPE_EINVAL;
  const int nk = s->dim == 3 ? 7 : 5;
  if (max < nk) return GPE_EINVAL;
  mask &= (1u << nk) - 1u;
  if (mask == 0) return GPE_EINVAL;
  static const char* n3[7] = {"flow_stage1", "flow_stage2", "flow_stage3", "ch_rk4_stage1",
                              "ch_rk4_stage2", "ch_rk4_stage3", "ch_rk4_stage4"};
  static const char* n2[5] = {"flow_stage1", "flow_stage2", "flow_stage3", "ch_rk2_stage1",
                              "ch_rk2_stage2"};
  // algorithmic HBM traffic per launch, in fields of one cell
  const double f3[7] = {9, 13, 16, 6, 8, 8, 7};
  const double f2[5] = {7, 10, 12, 5, 6};
  // all steps are enqueued back to back (no host synchronisation between
  // them), then read once
  KernelTimer proto;
  proto.mask = mask;
  // events of the boundaries in use only (the others stay null)
  std::vector<hipEvent_t> ev((size_t)nsteps * (nk + 1), nullptr);
  int rc = GPE_OK;
  for (size_t i = 0; i < ev.size() && rc == GPE_OK; ++i)
    if (proto.wants((int)(i % (size_t)(nk + 1))) && hipEventCreate(&ev[i]) != hipSuccess) rc = GPE_EHIP;
  std::vector<double> acc(nk, 0.0);
  for (int64_t st = 0; st < nsteps && rc == GPE_OK; ++st) {
    KernelTimer kt = proto;
    kt.ev = ev.data() + (size_t)st * (nk + 1);
    if (enqueue_step(s, &kt) != hipSuccess) { rc = GPE_EHIP; break; }
    s->step += 1;
  }
  if (rc == GPE_OK && hipStreamSynchronize(s->stream) != hipSuccess) rc = GPE_EHIP;
  for (int64_t st = 0; st < nsteps && rc == GPE_OK; ++st) {
    const hipEvent_t* e = ev.data() + (size_t)st * (nk + 1);
    for (int q = 0; q < nk; ++q) {
      if (!((mask >> q) & 1u)) continue;
      float t = 0;
      if (hipEventElapsedTime(&t, e[q], e[q + 1]) != hipSuccess) { rc = GPE_EHIP; break; }
      acc[q] += t;
    }
  }
  s->t = s->step * s->P.dt;
  for (auto& x : ev)
    if (x) (void)hipEventDestroy(x);
  if (rc) return rc;
  for (int q = 0; q < nk; ++q) {
    names[q] = s->dim == 3 ? n3[q] : n2[q];
    ms[q] = acc[q] / nsteps;
    bytes[q] = (s->dim == 3 ? f3[q] : f2[q]) * (double)s->ncell * (double)s->esize;
  }
  return nk;
}

int gpe_kernel_times(gpe_state* s, int64_t nsteps, int max, const char** names, double* ms, double* bytes) {
  return gpe_kernel_times_masked(s, nsteps, ~0u, max, names, ms, bytes);
}

void gpe_destroy(gpe_state* s) {
  if (!s) return;
  if (s->graph_ok) (void)hipGraphExecDestroy(s->graph);
  delete s;
}

const char* gpe_strerror(int code) {
  switch (code) {
    case GPE_OK: return "ok";
    case GPE_EINVAL: return "invalid argument";
    case GPE_EUNSTABLE: return "time step exceeds a linear stability estimate";
    case GPE_EWORKSPACE: return "workspace too small or misaligned";
    case GPE_EHIP: return "HIP runtime error";
    case GPE_ENONFINITE: return "state is not finite";
  }
  return "unknown error";
}

}  // extern "C"

// ---- experiment diagnostics --------------------------------------------------
namespace {

template <typename T>
gpe::PhaseArgs<T> phase_args(const gpe_state* s) {
  gpe::PhaseArgs<T> a;
  a.g = s->grid;
  a.axisym = s->axi ? 1 : 0;
  a.phi = buf<T>(s, B_PHI);
  for (int q = 0; q < 4; ++q) a.q[q] = buf<T>(s, B_Q0 + q);
  a.partial = buf<double>(s, B_SCR);
  a.result = a.partial + gpe::kDiagBlocks * 8;
  a.axis = 0;
  a.idx[0] = a.idx[1] = a.idx[2] = 0;
  return a;
}

// internal axis of problem axis a (2-D / axisymmetric grids are stored with
// the second axis as internal Z); -1 if the problem has no such axis
int internal_axis(const gpe_state* s, int a) {
  if (s->dim == 3) return (a >= 0 && a < 3) ? a : -1;
  return a == 0 ? 0 : (a == 1 ? 2 : -1);
}

int fetch_result(gpe_state* s, double out[8]) {
  const double* res = buf<double>(s, B_SCR) + gpe::kDiagBlocks * 8;
  if (hipMemcpyAsync(out, res, 8 * sizeof(double), hipMemcpyDeviceToHost, s->stream) != hipSuccess)
    return GPE_EHIP;
  if (hipStreamSynchronize(s->stream) != hipSuccess) return GPE_EHIP;
  return GPE_OK;
}

}  // namespace

extern "C" {

int gpe_phase_stats(gpe_state* s, double out[7]) {
  if (!s || !out) return GPE_EINVAL;
  const hipError_t e = s->P.precision == GPE_FP64 ? gpe::launch_phase_stats<double>(phase_args<double>(s), s->stream)
                                                  : gpe::launch_phase_stats<float>(phase_args<float>(s), s->stream);
  if (e != hipSuccess) return GPE_EHIP;
  double r[8];
  const int rc = fetch_result(s, r);
  if (rc) return rc;
  out[0] = r[0];
  for (int a = 0; a < 3; ++a) {
    const int ia = internal_axis(s, a);
    const bool ok = ia >= 0 && r[0] > 0.0;
    out[1 + a] = ok ? r[1 + ia] / r[0] : NAN;
    out[4 + a] = ok ? r[4 + ia] / r[0] : NAN;
  }
  return GPE_OK;
}

int gpe_interface_extent(gpe_state* s, double out[6]) {
  if (!s || !out) return GPE_EINVAL;
  const hipError_t e = s->P.precision == GPE_FP64
                           ? gpe::launch_interface_extent<double>(phase_args<double>(s), s->stream)
                           : gpe::launch_interface_extent<float>(phase_args<float>(s), s->stream);
  if (e != hipSuccess) return GPE_EHIP;
  double r[8];
  const int rc = fetch_result(s, r);
  if (rc) return rc;
  for (int a = 0; a < 3; ++a) {
    const int ia = internal_axis(s, a);
    const bool ok = ia >= 0 && std::isfinite(r[2 * ia]) && std::isfinite(r[2 * ia + 1]);
    out[2 * a] = ok ? -r[2 * ia] : NAN;
    out[2 * a + 1] = ok ? r[2 * ia + 1] : NAN;
  }
  return GPE_OK;
}

int gpe_line_crossings(gpe_state* s, int32_t axis, int32_t i0, int32_t i1, double out[2]) {
  if (!s || !out) return GPE_EINVAL;
  const int ia = internal_axis(s, axis);
  if (ia < 0) return GPE_EINVAL;
  // the other problem axes in increasing order get i0, i1
  int other[2], no = 0;
  for (int a = 0; a < s->dim; ++a)
    if (a != axis) other[no++] = a;
  const int32_t iv[2] = {i0, i1};
  int idx[3] = {0, 0, 0};
  for (int q = 0; q < 2; ++q) {
    if (q >= no) {
      if (iv[q] != 0) return GPE_EINVAL;
      continue;
    }
    const int io = internal_axis(s, other[q]);
    if (iv[q] < 0 || iv[q] >= s->grid.n[io]) return GPE_EINVAL;
    idx[io] = iv[q];
  }
  hipError_t e;
  if (s->P.precision == GPE_FP64) {
    gpe::PhaseArgs<double> a = phase_args<double>(s);
    a.axis = ia;
    for (int d = 0; d < 3; ++d) a.idx[d] = idx[d];
    e = gpe::launch_line_crossings<double>(a, s->stream);
  } else {
    gpe::PhaseArgs<float> a = phase_args<float>(s);
    a.axis = ia;
    for (int d = 0; d < 3; ++d) a.idx[d] = idx[d];
    e = gpe::launch_line_crossings<float>(a, s->stream);
  }
  if (e != hipSuccess) return GPE_EHIP;
  double r[8];
  const int rc = fetch_result(s, r);
  if (rc) return rc;
  out[0] = std::isfinite(r[0]) ? -r[0] : NAN;
  out[1] = std::isfinite(r[1]) ? r[1] : NAN;
  return GPE_OK;
}

}  // extern "C"
