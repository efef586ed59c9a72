// gpe_misc.hpp -- internal argument blocks of the initial-condition and
// diagnostics kernels.
#pragma once

#include <algorithm>

#include "gpe_device.hpp"

namespace gpe {

constexpr int kDiagBlocks = 512;

template <typename T>
struct InitArgs {
  int n[3];          // internal X, Y, Z sizes
  int pitch;         // elements per X row of a field (>= n[0])
  int kind;          // gpe_init_kind
  int has_y;         // 3-D: include the Y distance
  double center[3];  // internal axis order
  double radius, width, amp;
  T* phi;
  T* q[4];           // p, uX, uY, uZ (uY may be null)
};

template <typename T>
struct DiagArgs {
  Grid g;
  int axisym;
  double rho_l, rho_g;
  const T* phi;
  const T* q[4];     // p, uX, uY (null in 2-D), uZ
  double* partial;   // kDiagBlocks x 8
  double* result;    // 8
};

// Liquid-region moments and interface crossings (the experiment diagnostics)
template <typename T>
struct PhaseArgs {
  Grid g;
  int axisym;
  const T* phi;
  const T* q[4];     // p, uX, uY (null in 2-D), uZ
  double* partial;   // kDiagBlocks x 8
  double* result;    // 8
  // line crossings: internal axis and the indices of the two other axes
  int axis, idx[3];
};

template <typename T>
hipError_t launch_init(const InitArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_phase_stats(const PhaseArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_interface_extent(const PhaseArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_line_crossings(const PhaseArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_diag(const DiagArgs<T>& a, hipStream_t s);

}  // namespace gpe
