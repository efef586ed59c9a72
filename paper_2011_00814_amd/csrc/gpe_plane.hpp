// gpe_plane.hpp -- staging of one Z-plane of a work-group tile (with halo)
// from HBM into LDS, applying the boundary ghost rules while loading.
#pragma once

#include "gpe_device.hpp"

namespace gpe {

// In-plane addressing of the halo'd plane region [-2, PX-2) x [-2, PY-2) of a
// tile (relative to its first column x0 and row y0).  A tile whose region
// lies inside the domain ("interior") addresses every field at the plain
// cell offset with unit signs.  Other tiles map each position through the
// ghost rules: a cell-centred value, an X-face and a Y-face value get their
// own offsets, and the X-, Y- and Z-directed velocity components their
// in-plane signs.  The mapping depends on the in-plane position only, so it
// is computed once per work-group: per load pass the cell offset and one
// packed word holding the face offsets relative to it (which stay within a
// few cells) and the three signs.  A face whose sign is 0 (on a wall or
// symmetry plane) gets the cell offset, so every address stays in bounds.
template <typename T, int DIM, int PX, int PY, int NT>
struct PlaneMap {
  static constexpr int PLANE = PX * PY;
  static constexpr int NPASS = (PLANE + NT - 1) / NT;
  int off_c[NPASS];
  int pk[NPASS];  // boundary tiles: packed face deltas and signs
  bool ok[NPASS];
  bool interior;
  int x0, y0;

  struct Pos {
    int oc, ox, oy;  // in-plane offsets: cell value, X-face value, Y-face value
    T sx, sy, sz;    // in-plane signs of the X-, Y-, Z-directed components
  };

  __device__ __forceinline__ void init(const Grid& g, int x0_, int y0_) {
    x0 = x0_;
    y0 = y0_;
    const int nx = g.n[0], ny = g.n[1], pitch = g.pitch;
    interior = x0 - 2 >= 0 && x0 - 2 + PX - 1 <= nx - 1;
    if (DIM == 3) interior = interior && y0 - 2 >= 0 && y0 - 2 + PY - 1 <= ny - 1;
#pragma unroll
    for (int p = 0; p < NPASS; ++p) {
      const Pos q = map(g, p, ok[p]);
      off_c[p] = q.oc;
      // bits 0-7: X-face delta + 128, 8-15: Y-face delta in rows + 128,
      // 16-17 / 18-19 / 20-21: sx / sy / sz + 1
      const int dx = q.sx != T(0) ? q.ox - q.oc : 0;
      const int dy = q.sy != T(0) ? (q.oy - q.oc) / pitch : 0;
      pk[p] = (dx + 128) | ((dy + 128) << 8) | ((int)q.sx + 1) << 16 | ((int)q.sy + 1) << 18 |
              ((int)q.sz + 1) << 20;
    }
  }

  // full ghost-rule mapping of load pass p of this thread
  __device__ __forceinline__ Pos map(const Grid& g, int p, bool& ok_) const {
    const int nx = g.n[0], ny = g.n[1];
    const int lp = (int)threadIdx.x + p * NT;
    const int lx = lp % PX, ly = lp / PX;
    const int gx = x0 - 2 + lx;
    const int gy = (DIM == 3) ? y0 - 2 + ly : 0;
    Pos q{0, 0, 0, T(0), T(0), T(0)};
    ok_ = lp < PLANE && gx >= -2 && gx <= nx + 1;
    if (DIM == 3) ok_ = ok_ && gy >= -2 && gy <= ny + 1;
    if (!ok_) return q;
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
    q.oc = my * g.pitch + mx;
    q.ox = my * g.pitch + fx;
    q.oy = fy * g.pitch + mx;
    q.sx = T(fxs * wy);
    q.sy = T(fys * wx);
    q.sz = T(wx * wy);
    return q;
  }

  // false for positions of the outermost low halo row (ly = 0) in 3-D,
  // which only the phase field needs
  __device__ __forceinline__ bool inner_row(int p) const {
    if (DIM == 2) return true;
    const int lp = (int)threadIdx.x + p * NT;
    return lp >= PX;
  }

  // addressing of load pass p (valid when ok[p])
  __device__ __forceinline__ Pos pos(const Grid& g, int p) const {
    if (interior) return Pos{off_c[p], off_c[p], off_c[p], T(1), T(1), T(1)};
    const int w = pk[p], oc = off_c[p];
    const int dx = (w & 255) - 128, dy = ((w >> 8) & 255) - 128;
    return Pos{oc, oc + dx, oc + dy * g.pitch, T(((w >> 16) & 3) - 1), T(((w >> 18) & 3) - 1),
               T(((w >> 20) & 3) - 1)};
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
    const size_t pl = (size_t)g.pitch * g.n[1];
    zc = (size_t)mz * pl;
    zf = (size_t)fz * pl;
    tan = (rz == BC_WALL) ? T(-1) : T(1);
    nrm = T(fzs);
    r = T(mz) + T(0.5);
  }
};

}  // namespace gpe
