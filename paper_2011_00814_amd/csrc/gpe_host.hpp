// gpe_host.hpp -- host-side internals shared by the single-grid API
// (gpe_api.hip) and the batched ensemble (gpe_ensemble.hip).  Not part of
// the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "gpe.h"
#include "gpe_device.hpp"

namespace gpe_host {

// Workspace buffers of one grid (internal axis order for velocities: X, Y, Z).
enum Buf {
  B_Q0 = 0,   // p, uX, uY, uZ at time level n        (4 slots)
  B_Q1 = 4,   // first RK stage                       (4 slots)
  B_Q2 = 8,   // second RK stage                      (4 slots)
  B_PHI = 12, // phi*
  B_PHA = 13, // CH stage buffer A
  B_PHB = 14, // CH stage buffer B (RK4)
  B_ACC = 15, // running sum of the CH stage increments (RK2 and RK4)
  B_US = 16,  // u^n + u^{n+1} on X, Y, Z faces      (3 slots)
  B_SCR = 19, // reduction scratch
  B_COUNT = 20
};

constexpr size_t kAlign = 256;
constexpr size_t kRowAlign = 64;  // elements: every X row of a field starts on a 256-byte boundary

inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Elements from one X row of a field to the next.  FP32: the X extent
// rounded up to a multiple of kRowAlign (the padding is zero and never read),
// so the 32-column tile rows of the kernels start on a cache line; a grid
// narrower than kRowAlign keeps dense rows (a row then spans a cache line or
// two whatever its alignment).  FP64 keeps dense rows: a tile row there is
// two cache lines already, and padding measured no faster (0-3 % slower).
inline size_t row_pitch(const gpe_params* p) {
  const size_t nx = (size_t)p->n[0];
  if (p->precision == GPE_FP64 || nx < kRowAlign) return nx;
  return (nx + kRowAlign - 1) / kRowAlign * kRowAlign;
}

// Elements of one field buffer: rows of row_pitch for every (Y, Z) (2-D:
// every physical y; n[2] is 1 there).
inline size_t field_elems(const gpe_params* p) { return row_pitch(p) * (size_t)p->n[1] * (size_t)p->n[2]; }

}  // namespace gpe_host

struct gpe_state {
  gpe_params P;
  int dim;                 // 2 or 3
  bool axi;
  size_t esize;            // bytes per element
  size_t ncell;            // cells of the grid
  size_t fcell;            // elements of one field buffer (rows padded to grid.pitch)
  gpe::Grid grid;          // internal
  hipStream_t stream;
  char* ws;
  size_t ws_bytes;
  size_t off[gpe_host::B_COUNT];  // byte offsets; SIZE_MAX when absent
  int64_t step;
  double t;
  double mass_abs0;
  int sticky;
  hipGraphExec_t graph;
  bool graph_ok;
  int ncu;                 // compute units of the device the handle runs on
};

namespace gpe_host {

inline bool has_buf(const gpe_state* s, int b) { return s->off[b] != (size_t)-1; }

template <typename T>
T* buf(const gpe_state* s, int b) {
  return has_buf(s, b) ? reinterpret_cast<T*>(s->ws + s->off[b]) : nullptr;
}

// Kernel arguments of flow stage st (1..3) of a grid, with Z chunks of
// zchunk planes.
template <typename T>
gpe::FlowArgs<T> flow_args(const gpe_state* s, int st, int zchunk);

// Kernel arguments of the CH stages of one step (2 in 2-D / axisymmetric,
// 4 in 3-D) into a[] and their stage ids into stage[]; returns the count.
template <typename T>
int ch_args(const gpe_state* s, int zchunk, gpe::ChArgs<T> a[4], int stage[4]);

}  // namespace gpe_host
