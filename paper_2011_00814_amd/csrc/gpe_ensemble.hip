// gpe_ensemble.hip -- batched ensemble of independent 2-D / axisymmetric
// grids (include/gpe.h, "Batched ensemble").
//
// Every case is an ordinary grid handle (gpe_state) in its own slice of the
// caller's workspace, initialised by gpe_init_state.  The ensemble adds, in
// the head of the workspace, one argument block per case and stage (the
// same FlowArgs / ChArgs a single grid passes by value) and a table of
// work-group tiles over all cases.  A step is then five launches for the
// whole batch (three flow stages, two CH stages), each work-group reading
// its (case, tile) entry and that case's arguments; the five launches are
// captured once as a HIP graph and replayed.
//
// Tiles are TX columns x ZC rows (internal X x Z).  The table lists the
// tiles case by case and is permuted so that the round-robin dispatch of
// work-groups over the 8 XCDs gives each XCD a contiguous run of it: the
// tiles of one case share halo rows in the same L2.  Within a run the
// tallest tiles come first, so that a launch ends on short tiles.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "gpe.h"
#include "gpe_device.hpp"
#include "gpe_host.hpp"

namespace {

using gpe::ChArgs;
using gpe::FlowArgs;
using namespace gpe_host;

constexpr int kMaxCases = 65535;
constexpr int kEnsZChunk = 32;   // default rows per work-group tile of a case
constexpr int kMinZChunk = 1;    // smallest tile height (sizes the tile tables)
constexpr int kTuneRows[] = {1, 2, 4, 8, 16, 32, 64, 128};  // candidates of the autotuner
constexpr int kFinBlocks = 8;    // work-groups per case of the finite check

int clamp_rows(int rows, int nz) { return rows < nz ? rows : nz; }

// Byte layout of the workspace of a batch.
struct Layout {
  size_t flow_args, ch_args, flow_tiles, ch_tiles, flags, fields, ncell, total;
  std::vector<size_t> case_off, case_bytes;
  int max_flow_tiles = 0, max_ch_tiles = 0;  // table capacity
};

template <typename T>
bool make_layout(const gpe_params* c, int count, Layout& L) {
  L.case_off.assign(count, 0);
  L.case_bytes.assign(count, 0);
  long nft = 0, nct = 0;
  for (int i = 0; i < count; ++i) {
    const int nx = c[i].n[0], nz = c[i].n[1];  // internal X, Z of a 2-D grid
    const long zc = clamp_rows(kMinZChunk, nz);  // room for the most tiles any tile height gives
    nft += (long)((nx + gpe::FlowTile<2, T>::TX - 1) / gpe::FlowTile<2, T>::TX) * ((nz + zc - 1) / zc);
    nct += (long)((nx + gpe::ChTile<2, T>::TX - 1) / gpe::ChTile<2, T>::TX) * ((nz + zc - 1) / zc);
  }
  if (nft > (1L << 30) || nct > (1L << 30)) return false;
  L.max_flow_tiles = (int)nft;
  L.max_ch_tiles = (int)nct;
  size_t o = 0;
  L.flow_args = o;
  o += align_up(3 * (size_t)count * sizeof(FlowArgs<T>));
  L.ch_args = o;
  o += align_up(2 * (size_t)count * sizeof(ChArgs<T>));
  L.flow_tiles = o;
  o += align_up((size_t)nft * sizeof(int4));
  L.ch_tiles = o;
  o += align_up((size_t)nct * sizeof(int4));
  L.flags = o;
  o += align_up((size_t)count * sizeof(int32_t));
  L.fields = o;
  o += align_up((size_t)count * 4 * sizeof(void*));
  L.ncell = o;
  o += align_up((size_t)count * sizeof(int64_t));
  for (int i = 0; i < count; ++i) {
    L.case_off[i] = o;
    L.case_bytes[i] = align_up(gpe_workspace_bytes(&c[i]));
    o += L.case_bytes[i];
  }
  L.total = o;
  return true;
}

// Batch validity: every case valid on its own, 2-D or axisymmetric, and all
// of one precision and geometry.
int check_batch(const gpe_params* c, int count) {
  if (!c || count < 1 || count > kMaxCases) return GPE_EINVAL;
  for (int i = 0; i < count; ++i) {
    if (c[i].geometry != GPE_GEOM_2D && c[i].geometry != GPE_GEOM_AXISYM) return GPE_EINVAL;
    if (c[i].geometry != c[0].geometry || c[i].precision != c[0].precision) return GPE_EINVAL;
    if (c[i].ch_transport != GPE_CH_CONSERVATIVE) return GPE_EINVAL;
    if (gpe_workspace_bytes(&c[i]) == 0) return GPE_EINVAL;
  }
  return GPE_OK;
}

// Tallest tiles first within each XCD's run of a tile list (the runs that
// xcd_order below hands to the XCDs): a stable sort by the tile's row count,
// so the tiles of one case stay together.  The work-groups dispatched last on
// an XCD are then the shortest, and a launch does not end with a few tall
// tiles running on an otherwise idle XCD.
void tallest_first(std::vector<int4>& list, const std::vector<int>& zc, const std::vector<int>& nz) {
  const int nb = (int)list.size();
  const int per = nb / 8, rem = nb % 8;
  auto rows = [&](const int4& t) {
    const int left = nz[t.x] - t.w * zc[t.x];
    return left < zc[t.x] ? left : zc[t.x];
  };
  int o = 0;
  for (int x = 0; x < 8; ++x) {
    const int n = per + (x < rem ? 1 : 0);
    std::stable_sort(list.begin() + o, list.begin() + o + n,
                     [&](const int4& a, const int4& b) { return rows(a) > rows(b); });
    o += n;
  }
}

// XCD-contiguous order of a tile list (the host twin of tile_of_block):
// work-group b runs on XCD b % 8 and takes tile xcd * per + min(xcd, rem) + b / 8.
std::vector<int4> xcd_order(const std::vector<int4>& list) {
  const int nb = (int)list.size();
  const int per = nb / 8, rem = nb % 8;
  std::vector<int4> out(nb);
  for (int b = 0; b < nb; ++b) {
    const int xcd = b % 8, local = b / 8;
    out[b] = list[xcd * per + (xcd < rem ? xcd : rem) + local];
  }
  return out;
}

// per-case finite flags: set to 1, then cleared by any non-finite value
__global__ __launch_bounds__(256) void fill_flags_kernel(int32_t* flags, int n) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i < n) flags[i] = 1;
}

template <typename T>
__global__ __launch_bounds__(256) void finite_kernel(const T* const* fields, int count, const int64_t* ncell,
                                                     int32_t* flags) {
  const int cs = (int)blockIdx.x / kFinBlocks, part = (int)blockIdx.x % kFinBlocks;
  if (cs >= count) return;
  const int64_t n = ncell[cs];
  bool bad = false;
  for (int f = 0; f < 4; ++f) {
    const T* a = fields[4 * cs + f];
    if (!a) continue;
    for (int64_t q = (int64_t)part * blockDim.x + threadIdx.x; q < n; q += (int64_t)kFinBlocks * blockDim.x)
      bad |= !isfinite(a[q]);
  }
  if (bad) flags[cs] = 0;
}

}  // namespace

struct gpe_ensemble {
  int count;
  int precision;
  int geometry;
  hipStream_t stream;
  char* ws;
  std::vector<gpe_state*> cases;
  Layout L;
  std::vector<int> rows;            // tile height (Z chunk) of every case
  int nflow_tiles = 0, nch_tiles = 0;  // tiles in the current tables
  hipGraphExec_t graph;
  bool graph_ok;
};

namespace {

template <typename T>
hipError_t enqueue_batch_step(gpe_ensemble* e) {
  const FlowArgs<T>* fa = reinterpret_cast<const FlowArgs<T>*>(e->ws + e->L.flow_args);
  const ChArgs<T>* ca = reinterpret_cast<const ChArgs<T>*>(e->ws + e->L.ch_args);
  const int4* ft = reinterpret_cast<const int4*>(e->ws + e->L.flow_tiles);
  const int4* ct = reinterpret_cast<const int4*>(e->ws + e->L.ch_tiles);
  for (int st = 1; st <= 3; ++st) {
    hipError_t r = gpe::launch_flow_batch<T>(fa + (size_t)(st - 1) * e->count, ft, e->nflow_tiles, e->geometry, st,
                                             e->stream);
    if (r != hipSuccess) return r;
  }
  const int stages[2] = {gpe::CH_RK2_1, gpe::CH_RK2_2};
  for (int q = 0; q < 2; ++q) {
    hipError_t r = gpe::launch_ch_batch<T>(ca + (size_t)q * e->count, ct, e->nch_tiles, e->geometry, stages[q],
                                           e->stream);
    if (r != hipSuccess) return r;
  }
  return hipSuccess;
}

hipError_t enqueue_batch(gpe_ensemble* e) {
  return e->precision == GPE_FP64 ? enqueue_batch_step<double>(e) : enqueue_batch_step<float>(e);
}

template <typename T>
int upload_tables(gpe_ensemble* e) {
  const int n = e->count;
  std::vector<FlowArgs<T>> fa(3 * (size_t)n);
  std::vector<ChArgs<T>> ca(2 * (size_t)n);
  std::vector<int4> ft, ct;
  std::vector<const void*> fields(4 * (size_t)n, nullptr);
  std::vector<int64_t> ncell(n);
  std::vector<int> zcs(n), nzs(n);
  for (int i = 0; i < n; ++i) {
    const gpe_state* s = e->cases[i];
    const int nx = s->grid.n[0], nz = s->grid.n[2];
    const int zc = clamp_rows(e->rows[i], nz);
    zcs[i] = zc;
    nzs[i] = nz;
    for (int st = 1; st <= 3; ++st) fa[(size_t)(st - 1) * n + i] = flow_args<T>(s, st, zc);
    ChArgs<T> h[4];
    int stage[4];
    if (ch_args<T>(s, zc, h, stage) != 2) return GPE_EINVAL;
    ca[i] = h[0];
    ca[(size_t)n + i] = h[1];
    const int fx = (nx + gpe::FlowTile<2, T>::TX - 1) / gpe::FlowTile<2, T>::TX;
    const int hx = (nx + gpe::ChTile<2, T>::TX - 1) / gpe::ChTile<2, T>::TX;
    const int nbz = (nz + zc - 1) / zc;
    for (int bz = 0; bz < nbz; ++bz) {
      for (int bx = 0; bx < fx; ++bx) ft.push_back(make_int4(i, bx, 0, bz));
      for (int bx = 0; bx < hx; ++bx) ct.push_back(make_int4(i, bx, 0, bz));
    }
    fields[4 * (size_t)i + 0] = buf<T>(s, B_Q0);
    fields[4 * (size_t)i + 1] = buf<T>(s, B_Q0 + 1);
    fields[4 * (size_t)i + 2] = buf<T>(s, B_Q0 + 3);
    fields[4 * (size_t)i + 3] = buf<T>(s, B_PHI);
    ncell[i] = (int64_t)s->fcell;  // whole buffers: the row padding is zero
  }
  if ((int)ft.size() > e->L.max_flow_tiles || (int)ct.size() > e->L.max_ch_tiles) return GPE_EINVAL;
  e->nflow_tiles = (int)ft.size();
  e->nch_tiles = (int)ct.size();
  tallest_first(ft, zcs, nzs);
  tallest_first(ct, zcs, nzs);
  ft = xcd_order(ft);
  ct = xcd_order(ct);
  char* w = e->ws;
  const hipMemcpyKind h2d = hipMemcpyHostToDevice;
  if (hipMemcpyAsync(w + e->L.flow_args, fa.data(), fa.size() * sizeof(fa[0]), h2d, e->stream) != hipSuccess ||
      hipMemcpyAsync(w + e->L.ch_args, ca.data(), ca.size() * sizeof(ca[0]), h2d, e->stream) != hipSuccess ||
      hipMemcpyAsync(w + e->L.flow_tiles, ft.data(), ft.size() * sizeof(int4), h2d, e->stream) != hipSuccess ||
      hipMemcpyAsync(w + e->L.ch_tiles, ct.data(), ct.size() * sizeof(int4), h2d, e->stream) != hipSuccess ||
      hipMemcpyAsync(w + e->L.fields, fields.data(), fields.size() * sizeof(void*), h2d, e->stream) != hipSuccess ||
      hipMemcpyAsync(w + e->L.ncell, ncell.data(), ncell.size() * sizeof(int64_t), h2d, e->stream) != hipSuccess)
    return GPE_EHIP;
  if (hipStreamSynchronize(e->stream) != hipSuccess) return GPE_EHIP;
  return GPE_OK;
}

void destroy_cases(gpe_ensemble* e) {
  for (gpe_state* s : e->cases) gpe_destroy(s);
  e->cases.clear();
}

}  // namespace

extern "C" {

size_t gpe_ensemble_workspace_bytes(const gpe_params* cases, int32_t count) {
  if (check_batch(cases, count) != GPE_OK) return 0;
  Layout L;
  const bool ok = cases[0].precision == GPE_FP64 ? make_layout<double>(cases, count, L)
                                                 : make_layout<float>(cases, count, L);
  return ok ? L.total : 0;
}

int gpe_ensemble_create(const gpe_params* cases, int32_t count, void* d_workspace, size_t bytes,
                        void* hip_stream, gpe_ensemble** out) {
  if (!out) return GPE_EINVAL;
  *out = nullptr;
  int r = check_batch(cases, count);
  if (r) return r;
  gpe_ensemble* e = new (std::nothrow) gpe_ensemble();
  if (!e) return GPE_EINVAL;
  e->count = count;
  e->precision = cases[0].precision;
  e->geometry = cases[0].geometry;
  e->stream = (hipStream_t)hip_stream;
  e->ws = (char*)d_workspace;
  e->graph_ok = false;
  const bool ok = e->precision == GPE_FP64 ? make_layout<double>(cases, count, e->L)
                                           : make_layout<float>(cases, count, e->L);
  if (!ok) {
    delete e;
    return GPE_EINVAL;
  }
  if (!d_workspace || bytes < e->L.total || ((uintptr_t)d_workspace % kAlign) != 0) {
    delete e;
    return GPE_EWORKSPACE;
  }
  e->cases.reserve(count);
  for (int i = 0; i < count; ++i) {
    gpe_state* s = nullptr;
    r = gpe_init_state(&cases[i], e->ws + e->L.case_off[i], e->L.case_bytes[i], hip_stream, nullptr, nullptr, &s);
    if (r) {
      destroy_cases(e);
      delete e;
      return r;
    }
    e->cases.push_back(s);
  }
  e->rows.assign(count, kEnsZChunk);
  r = e->precision == GPE_FP64 ? upload_tables<double>(e) : upload_tables<float>(e);
  if (r) {
    destroy_cases(e);
    delete e;
    return r;
  }
  *out = e;
  return GPE_OK;
}

int gpe_ensemble_run_n(gpe_ensemble* e, int64_t nsteps) {
  if (!e || nsteps < 0) return GPE_EINVAL;
  if (nsteps == 0) return GPE_OK;
  if (e->stream == nullptr || nsteps < 2) {
    for (int64_t q = 0; q < nsteps; ++q)
      if (enqueue_batch(e) != hipSuccess) return GPE_EHIP;
  } else {
    if (!e->graph_ok) {
      hipGraph_t gr;
      if (hipStreamBeginCapture(e->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return GPE_EHIP;
      hipError_t r = enqueue_batch(e);
      hipError_t r2 = hipStreamEndCapture(e->stream, &gr);
      if (r != hipSuccess || r2 != hipSuccess) return GPE_EHIP;
      r = hipGraphInstantiate(&e->graph, gr, nullptr, nullptr, 0);
      (void)hipGraphDestroy(gr);
      if (r != hipSuccess) return GPE_EHIP;
      e->graph_ok = true;
    }
    for (int64_t q = 0; q < nsteps; ++q)
      if (hipGraphLaunch(e->graph, e->stream) != hipSuccess) return GPE_EHIP;
  }
  for (gpe_state* s : e->cases) {
    s->step += nsteps;
    s->t = s->step * s->P.dt;
  }
  return GPE_OK;
}

int gpe_ensemble_autotune(gpe_ensemble* e, int32_t trial_steps, int32_t* h_rows) {
  if (!e || trial_steps < 1 || e->stream == nullptr) return GPE_EINVAL;
  // size classes: cases with the same number of rows (internal Z)
  std::vector<int> classes;
  for (gpe_state* s : e->cases) {
    const int nz = s->grid.n[2];
    bool seen = false;
    for (int c : classes) seen = seen || c == nz;
    if (!seen) classes.push_back(nz);
  }
  hipEvent_t t0, t1;
  if (hipEventCreate(&t0) != hipSuccess) return GPE_EHIP;
  if (hipEventCreate(&t1) != hipSuccess) {
    (void)hipEventDestroy(t0);
    return GPE_EHIP;
  }
  int rc = GPE_OK;
  // time trial_steps batch steps with the current tables (re-uploaded and
  // re-captured); the steps advance every case
  auto trial = [&](float& ms) -> int {
    if (e->graph_ok) (void)hipGraphExecDestroy(e->graph);
    e->graph_ok = false;
    int r = e->precision == GPE_FP64 ? upload_tables<double>(e) : upload_tables<float>(e);
    if (r) return r;
    r = gpe_ensemble_run_n(e, 1);  // warm the new tiling (eager)
    if (r) return r;
    if (hipEventRecord(t0, e->stream) != hipSuccess) return GPE_EHIP;
    r = gpe_ensemble_run_n(e, trial_steps);
    if (r) return r;
    if (hipEventRecord(t1, e->stream) != hipSuccess || hipEventSynchronize(t1) != hipSuccess ||
        hipEventElapsedTime(&ms, t0, t1) != hipSuccess)
      return GPE_EHIP;
    return GPE_OK;
  };
  // coordinate search: one size class at a time, the others held fixed
  for (int nz : classes) {
    int best_rows = -1;
    float best = 0.0f;
    int last = -1;
    for (int cand : kTuneRows) {
      const int rows = clamp_rows(cand, nz);
      if (rows == last) continue;  // candidates beyond the grid height coincide
      last = rows;
      for (int i = 0; i < e->count; ++i)
        if (e->cases[i]->grid.n[2] == nz) e->rows[i] = rows;
      float ms = 0.0f;
      rc = trial(ms);
      if (rc) break;
      if (best_rows < 0 || ms < best) {
        best = ms;
        best_rows = rows;
      }
    }
    if (rc) break;
    for (int i = 0; i < e->count; ++i)
      if (e->cases[i]->grid.n[2] == nz) e->rows[i] = best_rows;
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (rc) return rc;
  if (e->graph_ok) (void)hipGraphExecDestroy(e->graph);
  e->graph_ok = false;
  rc = e->precision == GPE_FP64 ? upload_tables<double>(e) : upload_tables<float>(e);
  if (rc) return rc;
  if (h_rows)
    for (int i = 0; i < e->count; ++i) h_rows[i] = e->rows[i];
  return GPE_OK;
}

int gpe_ensemble_finite(gpe_ensemble* e, int32_t* h_flags) {
  if (!e || !h_flags) return GPE_EINVAL;
  int32_t* flags = reinterpret_cast<int32_t*>(e->ws + e->L.flags);
  hipLaunchKernelGGL(fill_flags_kernel, dim3((e->count + 255) / 256), dim3(256), 0, e->stream, flags, e->count);
  if (hipGetLastError() != hipSuccess) return GPE_EHIP;
  const unsigned blocks = (unsigned)e->count * kFinBlocks;
  if (e->precision == GPE_FP64) {
    hipLaunchKernelGGL((finite_kernel<double>), dim3(blocks), dim3(256), 0, e->stream,
                       reinterpret_cast<const double* const*>(e->ws + e->L.fields), e->count,
                       reinterpret_cast<const int64_t*>(e->ws + e->L.ncell), flags);
  } else {
    hipLaunchKernelGGL((finite_kernel<float>), dim3(blocks), dim3(256), 0, e->stream,
                       reinterpret_cast<const float* const*>(e->ws + e->L.fields), e->count,
                       reinterpret_cast<const int64_t*>(e->ws + e->L.ncell), flags);
  }
  if (hipGetLastError() != hipSuccess) return GPE_EHIP;
  if (hipMemcpyAsync(h_flags, flags, (size_t)e->count * sizeof(int32_t), hipMemcpyDeviceToHost, e->stream) !=
          hipSuccess ||
      hipStreamSynchronize(e->stream) != hipSuccess)
    return GPE_EHIP;
  return GPE_OK;
}

gpe_state* gpe_ensemble_case(gpe_ensemble* e, int32_t i) {
  if (!e || i < 0 || i >= e->count) return nullptr;
  return e->cases[i];
}

void gpe_ensemble_destroy(gpe_ensemble* e) {
  if (!e) return;
  if (e->graph_ok) (void)hipGraphExecDestroy(e->graph);
  destroy_cases(e);
  delete e;
}

}  // extern "C"
