// gpe_plane.hpp -- staging of one Z-plane of a work-group tile (with halo)
// from HBM into LDS, applying the boundary ghost rules while loading.
#pragma once

#include "gpe_device.hpp"

namespace gpe {

// Per-thread precomputed in-plane addressing of the halo'd plane region
// [-H, TX+H2) x [-H, TY+H2) of a tile (H = 2 low-side halo cells).  For each
// load pass the thread keeps the in-plane offset of a cell-centred value, of
// an X-face and of a Y-face value, and the in-plane signs of the X-, Y- and
// Z-directed velocity components.
template <typename T, int DIM, int PX, int PY, int NT>
struct PlaneMap {
  static constexpr int PLANE = PX * PY;
  static constexpr int NPASS = (PLANE + NT - 1) / NT;
  int off_c[NPASS], off_x[NPASS], off_y[NPASS];
  T sg_x[NPASS], sg_y[NPASS], sg_z[NPASS];
  bool ok[NPASS];

  __device__ __forceinline__ void init(const Grid& g, int x0, int y0) {
    const int nx = g.n[0], ny = g.n[1];
#pragma unroll
    for (int p = 0; p < NPASS; ++p) {
      const int lp = (int)threadIdx.x + p * NT;
      const int lx = lp % PX, ly = lp / PX;
      const int gx = x0 - 2 + lx;
      const int gy = (DIM == 3) ? y0 - 2 + ly : 0;
      bool ok_ = lp < PLANE && gx >= -2 && gx <= nx + 1;
      if (DIM == 3) ok_ = ok_ && gy >= -2 && gy <= ny + 1;
      ok[p] = ok_;
      off_c[p] = off_x[p] = off_y[p] = 0;
      sg_x[p] = sg_y[p] = sg_z[p] = T(0);
      if (!ok_) continue;
      int rx, ry = 0, fxs, fys = 1;
      const int mx = map_cell(gx, nx, g.bc[0], g.bc[1], rx);
      const int fx = map_face(gx, nx, g.bc[0], fxs);
      int my = 0, fy = 0;
      if (DIM == 3) {
        my = map_cell(gy, ny, g.bc[2], g.bc[3], ry);
        fy = map_face(gy, ny, g.bc[2], fys);
      }
      const int wx = (rx == BC_WALL) ? -1 : 1;
      const int wy = (ry == BC_WALL) ? -1 : 1;
      off_c[p] = my * nx + mx;
      off_x[p] = my * nx + fx;
      off_y[p] = fy * nx + mx;
      sg_x[p] = T(fxs * wy);
      sg_y[p] = T(fys * wx);
      sg_z[p] = T(wx * wy);
    }
  }
};

// Z-direction addressing of plane k (uniform across the work-group).
template <typename T>
struct ZMap {
  size_t zc, zf;  // element offsets of the mapped cell plane and face plane
  T tan;          // sign of X/Y velocity components (odd across a Z wall)
  T nrm;          // sign of the Z velocity component (0 on a Z boundary face)
  T r;            // radius of the mapped in-domain plane (axisymmetric: k + 1/2)
  __device__ __forceinline__ ZMap(const Grid& g, int k) {
    int rz, fzs;
    const int mz = map_cell(k, g.n[2], g.bc[4], g.bc[5], rz);
    const int fz = map_face(k, g.n[2], g.bc[4], fzs);
    const size_t pl = (size_t)g.n[0] * g.n[1];
    zc = (size_t)mz * pl;
    zf = (size_t)fz * pl;
    tan = (rz == BC_WALL) ? T(-1) : T(1);
    nrm = T(fzs);
    r = T(mz) + T(0.5);
  }
};

}  // namespace gpe
