// gpe_device.hpp -- internal types and device helpers shared by the kernels
// of libgpe (gfx950).  Not part of the public ABI.
//
// Internal axes: X (contiguous), Y (second in-plane axis, 3-D only) and Z,
// the axis every stencil kernel marches along.  2-D and axisymmetric grids
// are stored as (Z = physical y) x (X = physical x) with no Y axis, so one
// kernel template covers all three geometries: in axisymmetric geometry Z is
// the radial coordinate.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gpe {

enum { BC_PERIODIC = 0, BC_WALL = 1, BC_SYMMETRY = 2 };

// Grid description in internal axis order.  A field is stored as Z planes
// of Y rows; a row holds n[0] cells followed by unused padding up to pitch
// elements (FP32 from 64 cells on: a multiple of 64, so every row starts on
// a 256-byte boundary and the 32-column tile rows of the kernels cover whole
// cache lines; otherwise dense rows, pitch = n[0]).
struct Grid {
  int n[3];    // cells along X, Y, Z (n[1] = 1 in 2-D)
  int pitch;   // elements from one X row to the next (>= n[0])
  int bc[6];   // X-lo, X-hi, Y-lo, Y-hi, Z-lo, Z-hi
  int zchunk;  // output planes per work-group along Z
  int nb[3];   // work-group tiles along X, Y and Z chunks (set by the launcher)
};

// Work-groups of a 1-D launch are dispatched round-robin over the 8 XCDs
// (each with its own L2).  Give every XCD a contiguous run of the tile index
// (X fastest, then Y, then Z chunk) so that tiles sharing halo rows share an
// L2: tile = xcd * (nb / 8) + min(xcd, nb % 8) + (block / 8).
__device__ __forceinline__ void tile_of_block(const Grid& g, int& tx, int& ty, int& tz) {
  const int nb = g.nb[0] * g.nb[1] * g.nb[2];
  const int b = (int)blockIdx.x;
  const int xcd = b % 8, local = b / 8;
  const int per = nb / 8, rem = nb % 8;
  const int L = xcd * per + min(xcd, rem) + local;
  tx = L % g.nb[0];
  ty = (L / g.nb[0]) % g.nb[1];
  tz = L / (g.nb[0] * g.nb[1]);
}

// Constants in the working precision.
template <typename T>
struct Consts {
  T dt, cs2;
  T rho_l, rho_g, eta_l, eta_g;
  T sigma, mob;
  T a4;      // 4 a,  a = 3 / (4 W)
  T kappa6;  // 6 kappa, kappa = 3 W / 8
  T rho_ref;
  T g[3];    // body force, internal axis order
  T w1, w2, w3;  // lattice weights of links with 1, 2, 3 non-zero components
  // mixture laws as affine maps of the clamped phase field f:
  // rho = rho_a + 2 rho_hb f, eta = eta_a + eta_b f; hsig = -sigma / 2
  T rho_a, rho_hb, eta_a, eta_b, hsig;
};

template <typename T>
struct FlowArgs {
  Grid g;
  Consts<T> c;
  const T* src[4];  // stage input (p, uX, uY, uZ)
  const T* qn[4];   // time level n (read pointwise in stage 2)
  T* dst[4];        // stage output; in stage 3 also time level n (updated in place)
  const T* phi;     // frozen phase field
  T* usum[3];       // stage 3: u^n + u^{n+1} on each face family
  T* mu;            // FP64: mu of the frozen phi, written by stage 1 and read by stages 2 and 3
};

enum ChStage { CH_RK2_1 = 0, CH_RK2_2 = 1, CH_RK4_1 = 2, CH_RK4_2 = 3, CH_RK4_3 = 4, CH_RK4_4 = 5 };

template <typename T>
struct ChArgs {
  Grid g;
  Consts<T> c;
  const T* phi_in;  // phase field the RHS is evaluated on (read with halo 2)
  const T* usum[3]; // u^n + u^{n+1} on faces (centre velocity = 1/4 of the face pair sum)
  const T* phis;    // phi* (start of the sub-step), read pointwise
  T* acc;           // running sum of the increments: a (RK2), a + 2b + 2c + d (RK4)
  T* out;           // next stage input or the new phi*
  int adv;          // 1: convection u_hat . grad(phi); 0: div(phi u_hat)
};

// ---------------------------------------------------------------------------
// Ghost rules: walls, symmetry planes and the axis lie on cell faces.
// Cell-centred scalars are mirrored; the boundary-normal velocity is 0 on the
// boundary face and odd across it; tangential velocity is odd across a
// no-slip wall and even across a symmetry plane; periodic axes wrap.
// ---------------------------------------------------------------------------

// Cell index c (-2 <= c <= n+1) along an axis.  refl receives the BC of the
// mirror crossed (0 if none).
__device__ __forceinline__ int map_cell(int c, int n, int lo, int hi, int& refl) {
  refl = 0;
  if (c < 0) {
    if (lo == BC_PERIODIC) return c + n;
    refl = lo;
    return -1 - c;
  }
  if (c >= n) {
    if (hi == BC_PERIODIC) return c - n;
    refl = hi;
    return 2 * n - 1 - c;
  }
  return c;
}

// Face index f along its own normal axis.  sign becomes 0 for a boundary
// face, -1 for a mirrored face.  The returned index is always in range.
__device__ __forceinline__ int map_face(int f, int n, int lo, int& sign) {
  sign = 1;
  if (lo == BC_PERIODIC) {
    if (f < 0) return f + n;
    if (f >= n) return f - n;
    return f;
  }
  if (f <= 0) {
    if (f == 0) { sign = 0; return 0; }
    sign = -1;
    return -f;
  }
  if (f >= n) {
    if (f == n) { sign = 0; return 0; }
    sign = -1;
    return 2 * n - f;
  }
  return f;
}

template <typename T>
__device__ __forceinline__ T clamp1(T x) {
  return fmin(fmax(x, T(-1)), T(1));
}

// rho(phi) = [rho_L (1 + f) + rho_G (1 - f)] / 2 and likewise eta (f = phi
// clamped to [-1, 1]), evaluated as affine maps with host-precomputed
// coefficients.
template <typename T>
__device__ __forceinline__ T rho_of(const Consts<T>& c, T phi) {
  return fma(T(2) * c.rho_hb, clamp1(phi), c.rho_a);
}

template <typename T>
__device__ __forceinline__ T eta_of(const Consts<T>& c, T phi) {
  return fma(c.eta_b, clamp1(phi), c.eta_a);
}

// Element at a 32-bit in-plane offset from a work-group-uniform plane base.
// Written as base + zero-extended byte offset, so the access uses a scalar
// 64-bit base and one 32-bit vector offset instead of a per-thread 64-bit
// address (the library limits a plane to < 2^32 bytes).
template <typename T>
__device__ __forceinline__ T& at(T* plane, int off) {
  return *reinterpret_cast<T*>(reinterpret_cast<char*>(plane) + (uint32_t)off * (uint32_t)sizeof(T));
}
template <typename T>
__device__ __forceinline__ const T& at(const T* plane, int off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(plane) + (uint32_t)off * (uint32_t)sizeof(T));
}

// Element at a 32-bit byte offset from a work-group-uniform base.  Loop
// invariant offsets are passed through refresh() once per plane: the empty
// asm statement makes the value look updated in place, so the compiler can
// neither hoist a 64-bit zero-extended copy out of the plane loop nor keep
// a copy, and addresses each access as scalar base + 32-bit vector offset
// (no 64-bit vector add per access).
__device__ __forceinline__ void refresh(uint32_t& x) { asm volatile("" : "+v"(x)); }
template <typename T>
__device__ __forceinline__ const T& at_b(const T* base, uint32_t byte_off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}
template <typename T>
__device__ __forceinline__ T& at_b(T* base, uint32_t byte_off) {
  return *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byte_off);
}

// Streaming accesses for values read or written once per launch (the
// pointwise stage inputs and every output): non-temporal, so they do not
// displace the halo lines that neighbouring work-groups re-read from L2.
template <typename T>
__device__ __forceinline__ T ld_nt(const T* base, uint32_t byte_off) {
  return __builtin_nontemporal_load(&at_b(base, byte_off));
}
template <typename T>
__device__ __forceinline__ void st_nt(T* base, uint32_t byte_off, T v) {
  __builtin_nontemporal_store(v, &at_b(base, byte_off));
}

// Wave priority on its SIMD (0 lowest .. 3).  The stencil kernels raise it
// while a wave commits a staged plane to LDS and issues the next plane's
// global loads, keep it at 1 for the LDS-heavy derived fields and drop it to
// 0 for the arithmetic of the output, so that memory requests leave as early
// as possible while the other waves of the SIMD compute.  Raising it for the
// stores as well was slower.
template <int P>
__device__ __forceinline__ void wave_prio() {
  __builtin_amdgcn_s_setprio(P);
}

// Position (ex, ey) of index e in a W x H region of a staged LDS plane whose
// rows are longer than W.  Enumerated row by row, a 32-lane half-wave that
// crosses a row break skips the row's padding and hits two banks twice.  For
// 32 < W < 64 the first 32 H indices therefore run along rows of 32 columns
// (32 consecutive LDS words per half-wave) and the last W - 32 columns
// follow, interleaved across them.  Other shapes are enumerated row by row.
template <int W, int H>
__device__ __forceinline__ void region_pos(int e, int& ex, int& ey) {
  constexpr int X = W - 32;
  if (H == 1 || X <= 0 || X >= 32) {
    ex = e % W;
    ey = e / W;
  } else if (e < 32 * H) {
    ex = e & 31;
    ey = e >> 5;
  } else {
    const int t = e - 32 * H;
    ex = 32 + t % X;
    ey = t / X;
  }
}

// Reciprocal: hardware approximation (1 ulp) in FP32, exact division in FP64.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// Launchers (explicitly instantiated for float and double).
// scheme: gpe_scheme flags (non-zero ablation variants exist for 3-D only).
template <typename T>
hipError_t launch_flow(const FlowArgs<T>& a, int geometry, int stage, int scheme, hipStream_t s);
template <typename T>
hipError_t launch_ch(const ChArgs<T>& a, int geometry, int stage, hipStream_t s);
// Batches of 2-D / axisymmetric grids (geometry 0 / 1): one launch runs
// ntiles work-group tiles, tiles[b] = (case, btx, 0, btz) with the
// arguments cases[case] (both arrays in device memory).
template <typename T>
hipError_t launch_flow_batch(const FlowArgs<T>* cases, const int4* tiles, int ntiles, int geometry, int stage,
                             hipStream_t s);
template <typename T>
hipError_t launch_ch_batch(const ChArgs<T>* cases, const int4* tiles, int ntiles, int geometry, int stage,
                           hipStream_t s);

// Work-group tile shapes (X x Y columns, marched along Z) and the number of
// work-groups per CU their LDS footprint allows.  FP32 3-D tiles are 32 x 16
// (512 threads, halo area 1.29x the tile); FP64 3-D tiles are 32 x 8.
template <int DIM, typename T>
struct FlowTile;
template <typename T>
struct FlowTile<2, T> { static constexpr int TX = 64, TY = 1, BPC = 8; };
template <>
struct FlowTile<3, float> { static constexpr int TX = 32, TY = 8, BPC = 4; };
template <>
struct FlowTile<3, double> { static constexpr int TX = 32, TY = 8, BPC = 2; };

template <int DIM, typename T>
struct ChTile;
template <typename T>
struct ChTile<2, T> { static constexpr int TX = 64, TY = 1, BPC = 8; };
template <>
struct ChTile<3, float> { static constexpr int TX = 32, TY = 16, BPC = 3; };
template <>
struct ChTile<3, double> { static constexpr int TX = 32, TY = 8, BPC = 2; };

// Planes per work-group along Z.  The work-groups of a launch march their
// Z chunks in step, so neighbouring tiles share halo rows in L2.  The chunk
// count c is chosen to keep the CU slots busy: with W = tiles x c
// work-groups on S = CUs x groups-per-CU slots, the slot-time used,
// W / (S ceil(W / S)), times the share of staged planes that are output
// planes, zc / (zc + 3), is maximised over chunks of 8 to zmax planes.  On
// MI355X a launch of many shorter chunks (several rounds of work-groups that
// drift out of step) beats one round of long ones beyond 256^3: measured
// best at zmax = 64 planes for FP32 and 128 for FP64.
inline int choose_zchunk(const int n[3], int tx, int ty, int bpc, int ncu, int zmax) {
  const long tiles = (long)((n[0] + tx - 1) / tx) * ((n[1] + ty - 1) / ty);
  const long slots = (long)ncu * bpc;
  int best_zc = n[2];
  double best = -1.0;
  for (int c = 1; c <= n[2]; ++c) {
    const int zc = (n[2] + c - 1) / c;
    if (zc < 8 && c > 1) break;
    if (zc > zmax) continue;
    const long w = tiles * ((n[2] + zc - 1) / zc);
    const long rounds = (w + slots - 1) / slots;
    const double score = (double)w / (double)(slots * rounds) * zc / (zc + 3.0);
    if (score > best + 1e-12) {
      best = score;
      best_zc = zc;
    }
  }
  return best_zc;
}

}  // namespace gpe
