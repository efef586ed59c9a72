// gpe_misc.hip -- in-kernel initial condition and the diagnostics
// reductions (phase mass, kinetic energy, max |div u|, phi range, max |u|,
// finiteness).  Reductions accumulate in FP64 in both precisions, in a fixed
// partition and order, so results are bitwise reproducible.
#include "gpe_misc.hpp"

namespace gpe {

template <typename T>
__global__ __launch_bounds__(256) void init_kernel(InitArgs<T> a) {
  const size_t ncell = (size_t)a.n[0] * a.n[1] * a.n[2];
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncell;
       c += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(c % a.n[0]);
    const int j = (int)((c / a.n[0]) % a.n[1]);
    const int k = (int)(c / ((size_t)a.n[0] * a.n[1]));
    const size_t at = ((size_t)k * a.n[1] + j) * a.pitch + i;  // element of cell (i, j, k)
    const double x = i + 0.5, y = j + 0.5, z = k + 0.5;
    double ph = a.amp;
    if (a.kind == 1 || a.kind == 2) {
      const double dx = x - a.center[0], dy = y - a.center[1], dz = z - a.center[2];
      const double r = sqrt(dx * dx + (a.has_y ? dy * dy : 0.0) + dz * dz);
      const double d = (a.kind == 1) ? (a.radius - r) : (r - a.radius);
      ph = tanh(2.0 * d / a.width);
    } else if (a.kind == 3) {
      const double z0 = a.center[2] + a.amp * cos(2.0 * 3.14159265358979323846 * x / a.n[0]);
      ph = tanh(2.0 * (z - z0) / a.width);
    } else if (a.kind == 4) {
      // ellipse / ellipsoid: semi-axes R (1 + amp) along x, R (1 - amp) along
      // the second physical axis (internal Y in 3-D, Z in 2-D), R along z (3-D)
      const double sa = a.radius * (1.0 + a.amp), sb = a.radius * (1.0 - a.amp);
      const double ex = (x - a.center[0]) / sa;
      double rr;
      if (a.has_y) {
        const double ey = (y - a.center[1]) / sb, ez = (z - a.center[2]) / a.radius;
        rr = ex * ex + ey * ey + ez * ez;
      } else {
        const double ez = (z - a.center[2]) / sb;
        rr = ex * ex + ez * ez;
      }
      ph = tanh(2.0 * a.radius * (1.0 - sqrt(rr)) / a.width);
    }
    a.phi[at] = T(ph);
    for (int f = 0; f < 4; ++f)
      if (a.q[f]) a.q[f][at] = T(0);
  }
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

// slots: 0 mass, 1 sum|phi|, 2 ke, 3 max|div|, 4 min phi (stored negated as
// a max), 5 max phi, 6 max|u|, 7 non-finite count.
// Each wave takes whole grid rows (fixed j, k), rows strided over the launch:
// the row's coordinates, weights and ghost-mapped neighbour rows along Y and
// Z are wave-uniform, and the lanes stride along X (coalesced).
constexpr int kDiagThreads = 512;
template <typename T>
__global__ __launch_bounds__(kDiagThreads) void diag_partial_kernel(DiagArgs<T> a) {
  const Grid& g = a.g;
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  constexpr int NW = kDiagThreads / 64;
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  const size_t pitch = (size_t)g.pitch, plane = pitch * ny;
  const T* const uax[3] = {a.q[1], a.q[2], a.q[3]};
  double acc[8] = {0.0, 0.0, 0.0, 0.0, -INFINITY, -INFINITY, 0.0, 0.0};
  const int nrow = ny * nz;
  for (int row = blockIdx.x * NW + wv; row < nrow; row += gridDim.x * NW) {
    const int j = row % ny, k = row / ny;
    const double wr = a.axisym ? (k + 0.5) : 1.0;
    const size_t own = (size_t)k * plane + (size_t)j * pitch;
    // per axis: offset of the row holding the low neighbour cell (density at
    // the low face) and of the row holding the high face, with that face's
    // sign; along X both are the own row (the lane maps i itself)
    int refl, sy = 1, sz = 1;
    const size_t lo_row[3] = {own, (size_t)k * plane + (size_t)map_cell(j - 1, ny, g.bc[2], g.bc[3], refl) * pitch,
                              (size_t)map_cell(k - 1, nz, g.bc[4], g.bc[5], refl) * plane + (size_t)j * pitch};
    const size_t hi_row[3] = {own, (size_t)k * plane + (size_t)map_face(j + 1, ny, g.bc[2], sy) * pitch,
                              (size_t)map_face(k + 1, nz, g.bc[4], sz) * plane + (size_t)j * pitch};
    const double hi_sign[3] = {1.0, (double)sy, (double)sz};
    for (int i = lane; i < nx; i += 64) {
      const size_t c = own + i;
      const double ph = (double)a.phi[c];
      acc[0] += wr * ph;
      acc[1] += wr * fabs(ph);
      acc[4] = fmax(acc[4], -ph);
      acc[5] = fmax(acc[5], ph);
      bool fin = isfinite(ph) && isfinite((double)a.q[0][c]);
      const double rho_c = 0.5 * (a.rho_l * (1.0 + fmin(fmax(ph, -1.0), 1.0)) +
                                  a.rho_g * (1.0 - fmin(fmax(ph, -1.0), 1.0)));
      int sx = 1;
      const int il = map_cell(i - 1, nx, g.bc[0], g.bc[1], refl);
      const int ih = map_face(i + 1, nx, g.bc[0], sx);
      double div = 0.0;
      for (int ax = 0; ax < 3; ++ax) {
        if (!uax[ax]) continue;
        const double uf = (double)uax[ax][c];
        fin = fin && isfinite(uf);
        acc[6] = fmax(acc[6], fabs(uf));
        // density at the low face: mean of the two adjacent cells
        const double phl = (double)a.phi[lo_row[ax] + (ax == 0 ? il : i)];
        const double fl = fmin(fmax(phl, -1.0), 1.0);
        const double rho_l = 0.5 * (a.rho_l * (1.0 + fl) + a.rho_g * (1.0 - fl));
        const double rho_f = 0.5 * (rho_l + rho_c);
        const double wf = (a.axisym && ax == 2) ? (double)k : wr;
        acc[2] += 0.5 * rho_f * uf * uf * wf;
        // high face value for the divergence
        const double uh = (ax == 0 ? (double)sx : hi_sign[ax]) * (double)uax[ax][hi_row[ax] + (ax == 0 ? ih : i)];
        if (a.axisym && ax == 2)
          div += ((k + 1.0) * uh - (double)k * uf) / (k + 0.5);
        else
          div += uh - uf;
      }
      acc[3] = fmax(acc[3], fabs(div));
      if (!fin) acc[7] += 1.0;
    }
  }
  __shared__ double red[NW][8];
  double r[8];
  r[0] = wave_sum(acc[0]); r[1] = wave_sum(acc[1]); r[2] = wave_sum(acc[2]);
  r[3] = wave_max(acc[3]); r[4] = wave_max(acc[4]); r[5] = wave_max(acc[5]);
  r[6] = wave_max(acc[6]); r[7] = wave_sum(acc[7]);
  if (lane == 0)
    for (int s = 0; s < 8; ++s) red[wv][s] = r[s];
  __syncthreads();
  if (threadIdx.x == 0) {
    double o[8];
    for (int s = 0; s < 8; ++s) o[s] = red[0][s];
    for (int w = 1; w < NW; ++w) {
      o[0] += red[w][0]; o[1] += red[w][1]; o[2] += red[w][2];
      o[3] = fmax(o[3], red[w][3]); o[4] = fmax(o[4], red[w][4]);
      o[5] = fmax(o[5], red[w][5]); o[6] = fmax(o[6], red[w][6]);
      o[7] += red[w][7];
    }
    for (int s = 0; s < 8; ++s) a.partial[(size_t)blockIdx.x * 8 + s] = o[s];
  }
}

__global__ __launch_bounds__(64) void diag_final_kernel(const double* partial, int nblk, double* out) {
  // one wave: lane l folds partials l, l+64, ... in order, then a fixed tree
  const int l = threadIdx.x;
  double acc[8] = {0.0, 0.0, 0.0, 0.0, -INFINITY, -INFINITY, 0.0, 0.0};
  for (int b = l; b < nblk; b += 64) {
    const double* p = partial + (size_t)b * 8;
    acc[0] += p[0]; acc[1] += p[1]; acc[2] += p[2];
    acc[3] = fmax(acc[3], p[3]); acc[4] = fmax(acc[4], p[4]);
    acc[5] = fmax(acc[5], p[5]); acc[6] = fmax(acc[6], p[6]);
    acc[7] += p[7];
  }
  double r[8];
  r[0] = wave_sum(acc[0]); r[1] = wave_sum(acc[1]); r[2] = wave_sum(acc[2]);
  r[3] = wave_max(acc[3]); r[4] = wave_max(acc[4]); r[5] = wave_max(acc[5]);
  r[6] = wave_max(acc[6]); r[7] = wave_sum(acc[7]);
  if (l == 0)
    for (int s = 0; s < 8; ++s) out[s] = r[s];
}

// ---------------------------------------------------------------------------
// Experiment diagnostics (Sec. 4: the falling drop's centroid velocity and
// aspect ratio, the coalescing drops' radius / half length and centroid
// velocity, the Rayleigh-Taylor fronts).
// ---------------------------------------------------------------------------

// centre value of face component ax at cell (i, j, k): mean of its low and
// high faces, the high face by the ghost rule of the boundary it may lie on
template <typename T>
__device__ __forceinline__ double centre_velocity(const Grid& g, const T* u, int ax, int i, int j, int k) {
  const int ny = g.n[1];
  const size_t pitch = (size_t)g.pitch;
  const double lo = (double)u[((size_t)k * ny + j) * pitch + i];
  int hi[3] = {i, j, k};
  int sgn;
  hi[ax] = map_face(hi[ax] + 1, g.n[ax], g.bc[2 * ax], sgn);
  const double up = sgn * (double)u[((size_t)hi[2] * ny + hi[1]) * pitch + hi[0]];
  return 0.5 * (lo + up);
}

// slots over the cells with phi > 0, weight w = r = k + 1/2 (axisymmetric)
// or 1: 0 sum w, 1-3 sum w x_c (internal X, Y, Z), 4-6 sum w u_c
template <typename T>
__global__ __launch_bounds__(256) void phase_stats_kernel(PhaseArgs<T> a) {
  const Grid& g = a.g;
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const size_t ncell = (size_t)nx * ny * nz;
  double acc[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncell;
       c += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(c % nx);
    const int j = (int)((c / nx) % ny);
    const int k = (int)(c / ((size_t)nx * ny));
    if (!((double)a.phi[((size_t)k * ny + j) * g.pitch + i] > 0.0)) continue;
    const double w = a.axisym ? (k + 0.5) : 1.0;
    acc[0] += w;
    acc[1] += w * (i + 0.5);
    acc[2] += w * (j + 0.5);
    acc[3] += w * (k + 0.5);
    for (int ax = 0; ax < 3; ++ax)
      if (a.q[1 + ax]) acc[4 + ax] += w * centre_velocity(g, a.q[1 + ax], ax, i, j, k);
  }
  __shared__ double red[4][7];
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  for (int s = 0; s < 7; ++s) {
    const double r = wave_sum(acc[s]);
    if (lane == 0) red[wv][s] = r;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int s = 0; s < 7; ++s) {
      double o = red[0][s];
      for (int w = 1; w < (int)(blockDim.x / 64); ++w) o += red[w][s];
      a.partial[(size_t)blockIdx.x * 8 + s] = o;
    }
    a.partial[(size_t)blockIdx.x * 8 + 7] = 0.0;
  }
}

__global__ __launch_bounds__(64) void sum8_final_kernel(const double* partial, int nblk, double* out) {
  const int l = threadIdx.x;
  double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int b = l; b < nblk; b += 64)
    for (int s = 0; s < 8; ++s) acc[s] += partial[(size_t)b * 8 + s];
  for (int s = 0; s < 8; ++s) {
    const double r = wave_sum(acc[s]);
    if (l == 0) out[s] = r;
  }
}

// phi = 0 crossing between cell c (coordinate x0 = index + 1/2) and its
// neighbour one cell further along the axis, by linear interpolation
__device__ __forceinline__ bool crossing(double f0, double f1, double x0, double& pos) {
  if ((f0 > 0.0) == (f1 > 0.0)) return false;
  pos = x0 + f0 / (f0 - f1);
  return true;
}

// slots 2a / 2a+1: smallest / largest crossing along internal axis a, over
// all neighbour pairs inside the grid (smallest stored negated as a max)
template <typename T>
__global__ __launch_bounds__(256) void interface_extent_kernel(PhaseArgs<T> a) {
  const Grid& g = a.g;
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const size_t ncell = (size_t)nx * ny * nz;
  const size_t stride[3] = {1, (size_t)g.pitch, (size_t)g.pitch * ny};
  double acc[6] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY, -INFINITY, -INFINITY};
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncell;
       c += (size_t)gridDim.x * blockDim.x) {
    const int idx[3] = {(int)(c % nx), (int)((c / nx) % ny), (int)(c / ((size_t)nx * ny))};
    const size_t at = idx[0] + idx[1] * stride[1] + idx[2] * stride[2];
    const double f0 = (double)a.phi[at];
    for (int ax = 0; ax < 3; ++ax) {
      if (idx[ax] + 1 >= g.n[ax]) continue;
      double pos;
      if (crossing(f0, (double)a.phi[at + stride[ax]], idx[ax] + 0.5, pos)) {
        acc[2 * ax] = fmax(acc[2 * ax], -pos);
        acc[2 * ax + 1] = fmax(acc[2 * ax + 1], pos);
      }
    }
  }
  __shared__ double red[4][6];
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  for (int s = 0; s < 6; ++s) {
    const double r = wave_max(acc[s]);
    if (lane == 0) red[wv][s] = r;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int s = 0; s < 6; ++s) {
      double o = red[0][s];
      for (int w = 1; w < (int)(blockDim.x / 64); ++w) o = fmax(o, red[w][s]);
      a.partial[(size_t)blockIdx.x * 8 + s] = o;
    }
    a.partial[(size_t)blockIdx.x * 8 + 6] = -INFINITY;
    a.partial[(size_t)blockIdx.x * 8 + 7] = -INFINITY;
  }
}

__global__ __launch_bounds__(64) void max8_final_kernel(const double* partial, int nblk, double* out) {
  const int l = threadIdx.x;
  double acc[8];
  for (int s = 0; s < 8; ++s) acc[s] = -INFINITY;
  for (int b = l; b < nblk; b += 64)
    for (int s = 0; s < 8; ++s) acc[s] = fmax(acc[s], partial[(size_t)b * 8 + s]);
  for (int s = 0; s < 8; ++s) {
    const double r = wave_max(acc[s]);
    if (l == 0) out[s] = r;
  }
}

// one work-group: first and last crossing along the line parallel to
// internal axis a.axis through a.idx (the axis' own entry ignored);
// result[0] = -first, result[1] = last (-inf if none)
template <typename T>
__global__ __launch_bounds__(256) void line_crossings_kernel(PhaseArgs<T> a) {
  const Grid& g = a.g;
  const int ax = a.axis, n = g.n[ax];
  const size_t stride[3] = {1, (size_t)g.pitch, (size_t)g.pitch * g.n[1]};
  size_t base = 0;
  for (int d = 0; d < 3; ++d)
    if (d != ax) base += (size_t)a.idx[d] * stride[d];
  double lo = -INFINITY, hi = -INFINITY;
  for (int t = (int)threadIdx.x; t + 1 < n; t += (int)blockDim.x) {
    double pos;
    const size_t c = base + (size_t)t * stride[ax];
    if (crossing((double)a.phi[c], (double)a.phi[c + stride[ax]], t + 0.5, pos)) {
      lo = fmax(lo, -pos);
      hi = fmax(hi, pos);
    }
  }
  __shared__ double red[4][2];
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  lo = wave_max(lo);
  hi = wave_max(hi);
  if (lane == 0) {
    red[wv][0] = lo;
    red[wv][1] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double l0 = red[0][0], h0 = red[0][1];
    for (int w = 1; w < (int)(blockDim.x / 64); ++w) {
      l0 = fmax(l0, red[w][0]);
      h0 = fmax(h0, red[w][1]);
    }
    a.result[0] = l0;
    a.result[1] = h0;
  }
}

template <typename T>
hipError_t launch_init(const InitArgs<T>& a, hipStream_t s) {
  const size_t ncell = (size_t)a.n[0] * a.n[1] * a.n[2];
  const unsigned blocks = (unsigned)std::min<size_t>((ncell + 255) / 256, 16384);
  hipLaunchKernelGGL((init_kernel<T>), dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_diag(const DiagArgs<T>& a, hipStream_t s) {
  hipLaunchKernelGGL((diag_partial_kernel<T>), dim3(kDiagBlocks), dim3(kDiagThreads), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(64), 0, s, a.partial, kDiagBlocks, a.result);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_phase_stats(const PhaseArgs<T>& a, hipStream_t s) {
  hipLaunchKernelGGL((phase_stats_kernel<T>), dim3(kDiagBlocks), dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sum8_final_kernel, dim3(1), dim3(64), 0, s, a.partial, kDiagBlocks, a.result);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_interface_extent(const PhaseArgs<T>& a, hipStream_t s) {
  hipLaunchKernelGGL((interface_extent_kernel<T>), dim3(kDiagBlocks), dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(max8_final_kernel, dim3(1), dim3(64), 0, s, a.partial, kDiagBlocks, a.result);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_line_crossings(const PhaseArgs<T>& a, hipStream_t s) {
  hipLaunchKernelGGL((line_crossings_kernel<T>), dim3(1), dim3(256), 0, s, a);
  return hipGetLastError();
}

template hipError_t launch_phase_stats<float>(const PhaseArgs<float>&, hipStream_t);
template hipError_t launch_phase_stats<double>(const PhaseArgs<double>&, hipStream_t);
template hipError_t launch_interface_extent<float>(const PhaseArgs<float>&, hipStream_t);
template hipError_t launch_interface_extent<double>(const PhaseArgs<double>&, hipStream_t);
template hipError_t launch_line_crossings<float>(const PhaseArgs<float>&, hipStream_t);
template hipError_t launch_line_crossings<double>(const PhaseArgs<double>&, hipStream_t);
template hipError_t launch_init<float>(const InitArgs<float>&, hipStream_t);
template hipError_t launch_init<double>(const InitArgs<double>&, hipStream_t);
template hipError_t launch_diag<float>(const DiagArgs<float>&, hipStream_t);
template hipError_t launch_diag<double>(const DiagArgs<double>&, hipStream_t);

}  // namespace gpe
