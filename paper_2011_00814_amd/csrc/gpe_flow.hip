// gpe_flow.hip -- one TVD-RK3 stage of the pressure and momentum equations
// (arXiv 2011.00814, Sec. 3) as a single fused kernel.
//
// Work decomposition: a work-group owns TX x TY columns of cells and marches
// along Z through ZC output planes.  Each plane of p, u_X, u_Y, u_Z and phi
// is staged once from HBM into a 3-plane LDS ring (with the in-plane halo
// and the boundary ghost rules applied while loading); eta and nu are
// derived from the frozen phi as the plane is staged; div u and mu of the
// current plane are formed once in LDS.  mu depends on the frozen phi only:
// in FP64, stage 1 also stores it and stages 2 and 3 stage the stored field
// like the others (one plane behind them, which the single LDS plane of mu
// allows) instead of forming it again (in FP32 that was slower: stage 2 no
// faster, stage 3 8 % slower at the 128-register limit).  Each thread then
// evaluates the
// pressure RHS at its cell and the momentum RHS at the three low faces of
// its cell, applies the Shu-Osher combination of the stage and writes the
// result.  Stage 3 updates time level n in place and also writes the face
// velocity sums u^n + u^{n+1} used for the centre velocity of the CH step.
//
// The viscous shear terms use edge fluxes eta_edge (d_a u_b + d_b u_a): each
// edge of the staggered grid is evaluated once per plane into LDS (3 edge
// families in 3-D, 1 in 2-D) and every face takes differences of them.
//
// The plane loop is unrolled by three with ring slots counted from the tile
// start, so most LDS addresses are compile-time offsets from the thread's
// own position (the 2-plane rings of eta, nu and the edge fluxes alternate by
// plane parity).  The transverse pressure average of the in-plane faces is
// separable: its per-plane partial sums are carried in registers.  The next
// plane's global loads are issued before the current plane's stencil work
// (software pipelining).
#include <type_traits>

#include "gpe.h"
#include "gpe_plane.hpp"

namespace gpe {

// Occupancy target: 4 waves per SIMD in FP32 (<= 128 VGPRs): four
// work-groups of 256 threads per CU (32 x 8 tiles, 40 KB of LDS each), so a
// barrier holds 4 waves and the four groups interleave their phases; the
// FP64 kernel is left to the compiler's register allocation.
template <typename T>
struct FlowOcc { static constexpr int W = sizeof(T) == 4 ? 4 : 1; };

// One work-group tile (btx, bty) x Z chunk btz of the grid described by A.
// SCH: gpe_scheme flags (0 = the paper's scheme; the others are ablations
// that drop the transverse pressure average and / or the bulk viscosity).
template <typename T, int DIM, bool AXI, int STAGE, int TX, int TY, int SCH = 0>
__device__ __forceinline__ void flow_stage_tile(const FlowArgs<T>& A, int btx, int bty, int btz) {
  constexpr bool PAVG = (SCH & GPE_SCHEME_NO_PAVG) == 0;
  constexpr bool BULK = (SCH & GPE_SCHEME_NO_BULK) == 0;
  constexpr int NT = TX * TY;
  constexpr int PX = TX + 3;                  // in-plane X range [-2, TX]
  constexpr int PY = (DIM == 3) ? TY + 3 : 1;  // in-plane Y range [-2, TY]
  constexpr int PLANE = PX * PY;
  constexpr int EY = (DIM == 3) ? PX : 0;     // LDS stride of a +Y step
  // LDS: 3-plane rings (slot of plane k = (k - z0) mod 3), 2-plane rings
  // (slot = k & 1) and single-plane buffers
  constexpr int S_P = 0, S_UX = 3, S_UY = 6, S_UZ = 9, S_PH = 12;
  constexpr int S_ET = 15, S_NU = 17;    // eta, nu of planes k, k+1
  constexpr int S_EXZ = 19, S_EYZ = 21;  // edge fluxes between planes k-1|k and k|k+1
  constexpr int S_MU = 23, S_DV = 24, S_EXY = 25, NSLOT = 26;
  __shared__ T lds[NSLOT * PLANE];

  const Grid& g = A.g;
  const Consts<T>& c = A.c;
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2], pitch = g.pitch;
  const int tx = (int)threadIdx.x % TX, ty = (int)threadIdx.x / TX;
  const int x0 = btx * TX, y0 = bty * TY;
  const int z0 = btz * g.zchunk;
  __builtin_assume(z0 >= 0);  // lets the plane-index conditions of the staging fold
  const int z1 = min(z0 + g.zchunk, nz);
  const int i = x0 + tx, j = (DIM == 3) ? y0 + ty : 0;
  const bool active = i < nx && j < ny;
  const int ij = j * pitch + i;  // in-plane offset of the own column
  const int own = ((DIM == 3) ? (ty + 2) * PX : 0) + tx + 2;
  T* const L0 = lds + own;  // LDS base of the thread's own column

  PlaneMap<T, DIM, PX, PY, NT> pm;
  pm.init(g, x0, y0);

  // ---- plane staging: fetch() issues the global loads of plane k into
  // registers; commit() applies the ghost-rule signs and writes them, with
  // the derived eta and nu, into a ring slot.  No arithmetic touches a
  // loaded value before commit(), so the loads stay in flight while the
  // current plane is processed.
  constexpr int NP = PlaneMap<T, DIM, PX, PY, NT>::NPASS;
  struct Staged {  // one plane's loaded values, per load pass (m: mu of the plane below)
    T p[NP], x[NP], y[NP], z[NP], f[NP], m[NP];
  };
  constexpr bool MU_STORE = sizeof(T) == 8;  // stage 1 stores mu, stages 2 and 3 read it
  constexpr bool MU_STORED = MU_STORE && STAGE >= 2;
  Staged R;  // the plane in flight in the main loop
  // Every lane issues every load, so no branch separates the loads from the
  // waits for them: a position outside the mapped halo (never read) loads
  // the plane's first element instead, and on the outermost row, where p and
  // u are never read, an interior tile loads them from the next row (cache
  // lines fetched anyway) and a boundary tile from the mapped position.
  // byte offsets of every load pass within a plane (loop invariant):
  // phi at the cell, p and u_Z at the cell (outermost row: the next row),
  // u_X and u_Y at their faces
  uint32_t bo_f[NP], bo_c[NP], bo_x[NP], bo_y[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const auto q = pm.pos(g, p);
    const bool ok = pm.ok[p];
    const int oc = ok ? q.oc : 0;
    const int dq = (DIM == 3 && pm.interior && !pm.inner_row(p)) ? pitch : 0;
    bo_f[p] = (uint32_t)oc * (uint32_t)sizeof(T);
    bo_c[p] = (uint32_t)(oc + dq) * (uint32_t)sizeof(T);
    bo_x[p] = (uint32_t)((ok ? q.ox : 0) + dq) * (uint32_t)sizeof(T);
    bo_y[p] = (uint32_t)((ok ? q.oy : 0) + dq) * (uint32_t)sizeof(T);
  }
  // with_mu: also load mu of plane k - 1 (stages 2 and 3)
  auto fetch = [&](int k, Staged& r, bool with_mu) {
    const ZMap<T> z(g, k);
    const T* __restrict__ bp = A.src[0] + z.zc;
    const T* __restrict__ bx = A.src[1] + z.zc;
    const T* __restrict__ by = A.src[2] + z.zc;
    const T* __restrict__ bz = A.src[3] + z.zf;
    const T* __restrict__ bf = A.phi + z.zc;
    const T* __restrict__ bm = A.mu;
    if (MU_STORED && with_mu) bm += ZMap<T>(g, k - 1).zc;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      refresh(bo_f[p]);
      refresh(bo_c[p]);
      refresh(bo_x[p]);
      if (DIM == 3) refresh(bo_y[p]);
      r.f[p] = at_b(bf, bo_f[p]);
      r.p[p] = at_b(bp, bo_c[p]);
      r.x[p] = at_b(bx, bo_x[p]);
      r.y[p] = (DIM == 3) ? at_b(by, bo_y[p]) : T(0);
      r.z[p] = at_b(bz, bo_c[p]);
      if (MU_STORED && with_mu) r.m[p] = at_b(bm, bo_f[p]);
    }
  };
  auto commit = [&](int s, int k, const Staged& r, bool with_mu) {
    const ZMap<T> z(g, k);
    T* const e2 = lds + (k & 1) * PLANE;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const int lp = (int)threadIdx.x + p * NT;
      if (lp >= PLANE) continue;
      const auto q = pm.pos(g, p);  // signs (all +1 inside an interior tile)
      const T ph = r.f[p];
      const T eta = eta_of(c, ph);
      lds[(S_P + s) * PLANE + lp] = r.p[p];
      lds[(S_UX + s) * PLANE + lp] = r.x[p] * (q.sx * z.tan);
      if (DIM == 3) lds[(S_UY + s) * PLANE + lp] = r.y[p] * (q.sy * z.tan);
      lds[(S_UZ + s) * PLANE + lp] = r.z[p] * (q.sz * z.nrm);
      lds[(S_PH + s) * PLANE + lp] = ph;
      e2[S_ET * PLANE + lp] = eta;
      e2[S_NU * PLANE + lp] = eta * recip(rho_of(c, ph));
      if (MU_STORED && with_mu) lds[S_MU * PLANE + lp] = r.m[p];
    }
  };

  // ---- chemical potential at an LDS position of plane k, given its phi
  // planes k, k-1, k+1 (Sec. 2, Sec. 3 isotropic Laplacian):
  // mu = 4 a phi (phi^2 - 1) - 6 kappa sum_i w_i (phi_i - phi_c)
  auto mu_at = [&](int k, const T* F0, const T* Fm, const T* Fp) -> T {
    const T f = F0[0];
    T rp = T(1), rm = T(1);
    if (AXI) {  // Z is radial: weight every link by its mid-point radius / r_k
      const T rk = T(k) + T(0.5);
      const T ir = T(1) / rk;
      rp = (rk + T(0.5)) * ir;
      rm = (rk - T(0.5)) * ir;
    }
    T lap;
    if (DIM == 2) {
      const T s1 = ((F0[1] - f) + (F0[-1] - f)) + (rp * (Fp[0] - f) + rm * (Fm[0] - f));
      const T s2 = rp * ((Fp[1] - f) + (Fp[-1] - f)) + rm * ((Fm[1] - f) + (Fm[-1] - f));
      lap = c.w1 * s1 + c.w2 * s2;
    } else {
      const T s1 = ((F0[1] - f) + (F0[-1] - f)) + ((F0[EY] - f) + (F0[-EY] - f)) +
                   ((Fp[0] - f) + (Fm[0] - f));
      lap = c.w1 * s1;
      if (c.w2 != T(0)) {
        const T s2 = ((F0[1 + EY] - f) + (F0[1 - EY] - f) + (F0[-1 + EY] - f) + (F0[-1 - EY] - f)) +
                     ((Fp[1] - f) + (Fp[-1] - f) + (Fp[EY] - f) + (Fp[-EY] - f)) +
                     ((Fm[1] - f) + (Fm[-1] - f) + (Fm[EY] - f) + (Fm[-EY] - f));
        lap += c.w2 * s2;
      }
      if (c.w3 != T(0)) {
        const T s3 = ((Fp[1 + EY] - f) + (Fp[1 - EY] - f) + (Fp[-1 + EY] - f) + (Fp[-1 - EY] - f)) +
                     ((Fm[1 + EY] - f) + (Fm[1 - EY] - f) + (Fm[-1 + EY] - f) + (Fm[-1 - EY] - f));
        lap += c.w3 * s3;
      }
    }
    return c.a4 * f * (f * f - T(1)) - c.kappa6 * lap;
  };

  // ---- velocity divergence at an LDS position of plane k (Sec. 3 div
  // stencil); axisymmetric: (1/r) d(r u_r)/dr with face radii k and k+1
  auto div_at = [&](int k, const T* UX, const T* UY, const T* UZ0, const T* UZp) -> T {
    T d = UX[1] - UX[0];
    if (DIM == 3) d += UY[EY] - UY[0];
    if (AXI) {
      const T rk = T(k) + T(0.5);
      d += ((T(k) + T(1)) * UZp[0] - T(k) * UZ0[0]) / rk;
    } else {
      d += UZp[0] - UZ0[0];
    }
    return d;
  };

  // ---- separable part of the transverse pressure average of an in-plane
  // face (normal offset ea, other in-plane axis eb) on one plane,
  // difference-first: 4 D_0 + D_{+b} + D_{-b} with D = p - p_{-a}
  auto prow = [&](const T* P, int ea, int eb) -> T {
    if (DIM == 2) return P[0] - P[-ea];
    return T(4) * (P[0] - P[-ea]) + ((P[eb] - P[eb - ea]) + (P[-eb] - P[-eb - ea]));
  };

  // ---- shear edge fluxes (Sec. 3 viscous stencils with the four-cell
  // average of eta on an edge, kept as the four-cell sum: the face stencils
  // carry the factor 1/4).  edge_z: edge between planes k and k+1 on the low
  // face along in-plane axis A (offset ea) of the cell at the pointers'
  // position: eta4 (d_z u_A + d_A u_Z).  edge_xy: edge at the low-X, low-Y
  // corner of the cell on plane k: eta4 (d_Y u_X + d_X u_Y).
  auto edge_z = [&](const T* UA0, const T* UAp, const T* UZp, const T* E0, const T* Ep, int ea) -> T {
    const T e4 = (E0[0] + Ep[0]) + (E0[-ea] + Ep[-ea]);
    return e4 * ((UAp[0] - UA0[0]) + (UZp[0] - UZp[-ea]));
  };
  auto edge_xy = [&](const T* UX0, const T* UY0, const T* E0) -> T {
    const T e4 = (E0[0] + E0[-EY]) + (E0[-1] + E0[-1 - EY]);
    return e4 * ((UX0[0] - UX0[-EY]) + (UY0[0] - UY0[-1]));
  };
  // edge fluxes of the Z-directed edges between planes k and k+1 (ring slots
  // s0, sp of the 3-plane rings) on positions [0, T] of the tile, into the
  // edge slot of plane k; with the in-plane edges of plane k when xy is set.
  // The region has a few positions more than the work-group has threads; the
  // thread index is rotated by one wave so that this loop's extra positions
  // fall to the second wave and those of the mu / div loop to the first.
  auto edges = [&](int k, int s0, int sp, bool xy) {
    constexpr int EN = (DIM == 3) ? (TX + 1) * (TY + 1) : TX + 1;
    constexpr int ROT = NT > 64 ? NT - 64 : 0;
    const int e0 = (k & 1) * PLANE, e1 = PLANE - e0;
    for (int e = ((int)threadIdx.x + ROT) % NT; e < EN; e += NT) {
      int ex, ey;
      region_pos<TX + 1, (DIM == 3) ? TY + 1 : 1>(e, ex, ey);
      const int q = ((DIM == 3) ? (ey + 2) * PX : 0) + ex + 2;
      T* d = lds + q;
      const T* E0 = d + S_ET * PLANE + e0;
      const T* Ep = d + S_ET * PLANE + e1;
      d[S_EXZ * PLANE + e0] = edge_z(d + (S_UX + s0) * PLANE, d + (S_UX + sp) * PLANE, d + (S_UZ + sp) * PLANE, E0, Ep, 1);
      if (DIM == 3) {
        d[S_EYZ * PLANE + e0] =
            edge_z(d + (S_UY + s0) * PLANE, d + (S_UY + sp) * PLANE, d + (S_UZ + sp) * PLANE, E0, Ep, EY);
        if (xy) d[S_EXY * PLANE] = edge_xy(d + (S_UX + s0) * PLANE, d + (S_UY + s0) * PLANE, E0);
      }
    }
  };

  // -------- warm-up: planes z0-2, z0-1, z0 into slots 1, 2, 0 -------------
  // (the ring slot of plane k is (k - z0) mod 3).  The loads of all three
  // are issued before the first is committed, so the warm-up waits for one
  // memory latency, not three.
  {
    Staged W0, W1, W2;
    fetch(z0 - 2, W0, false);
    fetch(z0 - 1, W1, false);
    fetch(z0, W2, true);  // with mu of plane z0 - 1
    commit(1, z0 - 2, W0, false);
    commit(2, z0 - 1, W1, false);
    commit(0, z0, W2, true);
  }
  __syncthreads();
  edges(z0 - 1, 2, 0, false);  // Z-directed edges between planes z0-1 and z0
  // eta and nu of the own cell on the previous plane (carried from plane to plane)
  T eta_prev = L0[S_ET * PLANE + ((z0 - 1) & 1) * PLANE];
  T nu_prev = L0[S_NU * PLANE + ((z0 - 1) & 1) * PLANE];
  T mu_prev = MU_STORED ? L0[S_MU * PLANE]
                        : mu_at(z0 - 1, L0 + (S_PH + 2) * PLANE, L0 + (S_PH + 1) * PLANE, L0 + (S_PH + 0) * PLANE);
  T dv_prev = div_at(z0 - 1, L0 + (S_UX + 2) * PLANE, L0 + (S_UY + 2) * PLANE, L0 + (S_UZ + 2) * PLANE,
                     L0 + (S_UZ + 0) * PLANE);
  T gx_m = prow(L0 + (S_P + 2) * PLANE, 1, EY), gx_0 = prow(L0 + (S_P + 0) * PLANE, 1, EY);
  T gy_m = T(0), gy_0 = T(0);
  if (DIM == 3) {
    gy_m = prow(L0 + (S_P + 2) * PLANE, EY, 1);
    gy_0 = prow(L0 + (S_P + 0) * PLANE, EY, 1);
  }
  fetch(z0 + 1, R, true);

  // time level n at the thread's own cell (stages 2 and 3), loaded at the
  // top of the plane's step (before the next plane's loads, so that waiting
  // for it in the update does not also wait for those)
  uint32_t bo_own = (uint32_t)(active ? ij : 0) * (uint32_t)sizeof(T);
  auto fetch_qn = [&](int k, T* dst) {
    refresh(bo_own);
    if (STAGE >= 2) {  // an inactive lane loads the plane's first element (unused)
      const size_t pk = (size_t)k * ny * pitch;
#pragma unroll
      for (int f = 0; f < 4; ++f)
        if (DIM == 3 || f != 2) dst[f] = ld_nt((STAGE == 3 ? A.dst[f] : A.qn[f]) + pk, bo_own);
    }
  };

  const T dt = c.dt;

  // one output plane k; planes k, k-1, k+1 sit in ring slots S0, SM, SP
  auto step = [&](auto slots, int k) {
    constexpr int S0 = decltype(slots)::value;
    constexpr int SM = (S0 + 2) % 3, SP = (S0 + 1) % 3;
    __syncthreads();  // readers of slot SP (plane k-2) and of mu (plane k-1) are done
    wave_prio<3>();
    commit(SP, k + 1, R, true);  // with mu of plane k
    T qn_cur[4] = {T(0), T(0), T(0), T(0)};
    fetch_qn(k, qn_cur);
    // in flight during this plane's work; the chunk's last plane loads plane
    // k + 1 again (just loaded, unused) so that the loads are unconditional
    fetch(k + 1 < z1 ? k + 2 : k + 1, R, true);
    wave_prio<0>();
    __syncthreads();
    wave_prio<1>();

    // div u and mu (unless staged) of plane k on [-1, T-1] (LDS positions 1 .. T+1)
    {
      constexpr int EN = (DIM == 3) ? (TX + 1) * (TY + 1) : TX + 1;
      for (int e = (int)threadIdx.x; e < EN; e += NT) {
        int ex, ey;
        region_pos<TX + 1, (DIM == 3) ? TY + 1 : 1>(e, ex, ey);
        const int q = ((DIM == 3) ? (ey + 1) * PX : 0) + ex + 1;
        T* b = lds + q;
        if (!MU_STORED)
          b[S_MU * PLANE] = mu_at(k, b + (S_PH + S0) * PLANE, b + (S_PH + SM) * PLANE, b + (S_PH + SP) * PLANE);
        b[S_DV * PLANE] = div_at(k, b + (S_UX + S0) * PLANE, b + (S_UY + S0) * PLANE,
                                 b + (S_UZ + S0) * PLANE, b + (S_UZ + SP) * PLANE);
      }
    }
    edges(k, S0, SP, true);
    wave_prio<0>();
    // pressure-average partial sums of plane k+1 (own column)
    const T gx_p = prow(L0 + (S_P + SP) * PLANE, 1, EY);
    T gy_p = T(0);
    if (DIM == 3) gy_p = prow(L0 + (S_P + SP) * PLANE, EY, 1);
    __syncthreads();

    if (active) {
      const T* P0 = L0 + (S_P + S0) * PLANE;
      const T* Pm = L0 + (S_P + SM) * PLANE;
      const T* Pp = L0 + (S_P + SP) * PLANE;
      const T* UX0 = L0 + (S_UX + S0) * PLANE;
      const T* UXm = L0 + (S_UX + SM) * PLANE;
      const T* UXp = L0 + (S_UX + SP) * PLANE;
      const T* UY0 = L0 + (S_UY + S0) * PLANE;
      const T* UYm = L0 + (S_UY + SM) * PLANE;
      const T* UYp = L0 + (S_UY + SP) * PLANE;
      const T* UZ0 = L0 + (S_UZ + S0) * PLANE;
      const T* UZm = L0 + (S_UZ + SM) * PLANE;
      const T* UZp = L0 + (S_UZ + SP) * PLANE;
      const T* PH0 = L0 + (S_PH + S0) * PLANE;
      const T* PHm = L0 + (S_PH + SM) * PLANE;
      const int e0 = (k & 1) * PLANE, e1 = PLANE - e0;  // 2-plane ring slots of k, k+1 (and k-1)
      const T* ET0 = L0 + S_ET * PLANE + e0;
      const T* NU0 = L0 + S_NU * PLANE + e0;
      const T* NUp = L0 + S_NU * PLANE + e1;
      const T* XZp = L0 + S_EXZ * PLANE + e0;  // edges between planes k and k+1
      const T* XZm = L0 + S_EXZ * PLANE + e1;  // edges between planes k-1 and k
      const T* YZp = L0 + S_EYZ * PLANE + e0;
      const T* YZm = L0 + S_EYZ * PLANE + e1;
      const T* XY = L0 + S_EXY * PLANE;
      const T* MU = L0 + S_MU * PLANE;
      const T* DV = L0 + S_DV * PLANE;

      // axisymmetric radii of row k (Z radial): centre r_k, faces R_k = k, R_{k+1}
      const T rk = T(k) + T(0.5);
      const T Rk = T(k), Rk1 = T(k) + T(1);
      const T inv_rk = T(1) / rk;

      // ---- pressure equation at the cell centre:
      // dp/dt = -rho cs^2 D + sum [nu_{+1/2} (p_+ - p) - nu_{-1/2} (p - p_-)]
      const T pc = P0[0], nuc = NU0[0];
      T diff = (nuc + NU0[1]) * (P0[1] - pc) - (nuc + NU0[-1]) * (pc - P0[-1]);
      if (DIM == 3) diff += (nuc + NU0[EY]) * (P0[EY] - pc) - (nuc + NU0[-EY]) * (pc - P0[-EY]);
      {
        const T fp = (nuc + NUp[0]) * (Pp[0] - pc);
        const T fm = (nuc + nu_prev) * (pc - Pm[0]);
        diff += AXI ? (Rk1 * fp - Rk * fm) * inv_rk : fp - fm;
      }
      const T fc = clamp1(PH0[0]);
      const T Lp = -fma(T(2) * c.rho_hb, fc, c.rho_a) * c.cs2 * DV[0] + T(0.5) * diff;

      // ---- momentum at an in-plane face (normal A with LDS offset ea, other
      // in-plane axis B with offset eb in 3-D, Z transverse) ----
      auto face_inplane = [&](const T* UA0, const T* UAm, const T* UAp, const T* UB0, int ea, int eb,
                              const T* EZp, const T* EZm, const T* EB, T gA, T gm, T g0, T gp) -> T {
        const T ua = UA0[0];
        const T phc = PH0[0], phl = PH0[-ea];
        const T rho_f = fma(c.rho_hb, fc + clamp1(phl), c.rho_a);  // mean of the two cells
        const T eh = ET0[0], el = ET0[-ea];
        // twice the convection: u d_a u + ubar_b d_b u + ubar_z d_z u
        T conv = ua * (UA0[ea] - UA0[-ea]);
        {
          const T sz = (UZ0[0] + UZ0[-ea]) + (UZp[0] + UZp[-ea]);
          T tr = sz * (UAp[0] - UAm[0]);
          if (DIM == 3) {
            const T sb = (UB0[0] + UB0[-ea]) + (UB0[eb] + UB0[eb - ea]);
            tr += sb * (UA0[eb] - UA0[-eb]);
          }
          conv += T(0.25) * tr;
        }
        // viscous stress divergence with edge-averaged eta, bulk eta_b = eta:
        // normal part, then the shear edge fluxes across Z and across B
        T V = T(2) * (eh * (UA0[ea] - ua) - el * (ua - UA0[-ea]));
        T Vt = AXI ? (Rk1 * EZp[0] - Rk * EZm[0]) * inv_rk : EZp[0] - EZm[0];
        if (DIM == 3) Vt += EB[eb] - EB[0];
        const T Vb = BULK ? eh * DV[0] - el * DV[-ea] : T(0);  // bulk viscosity eta_b = eta
        V += T(0.25) * Vt + Vb;
        // transversely averaged pressure gradient from the carried partial sums
        const T G = PAVG ? (T(4) * g0 + (gp + gm)) * (DIM == 2 ? T(1.0 / 6.0) : T(1.0 / 36.0))
                         : P0[0] - P0[-ea];
        const T S = c.hsig * (phc + phl) * (MU[0] - MU[-ea]);
        const T B = (rho_f - c.rho_ref) * gA;
        return fma(T(-0.5), conv, (-G + V + S + B) * recip(rho_f));
      };

      const T LuX = face_inplane(UX0, UXm, UXp, UY0, 1, EY, XZp, XZm, XY, c.g[0], gx_m, gx_0, gx_p);
      T LuY = T(0);
      if (DIM == 3) LuY = face_inplane(UY0, UYm, UYp, UX0, EY, 1, YZp, YZm, XY, c.g[1], gy_m, gy_0, gy_p);

      // ---- momentum at the Z face between planes k-1 and k ----
      T LuZ = T(0);
      const bool bZ = (k == 0 && g.bc[4] != BC_PERIODIC);
      if (!bZ) {
        const T uz = UZ0[0];
        const T phc = PH0[0], phl = PHm[0];
        const T rho_f = fma(c.rho_hb, fc + clamp1(phl), c.rho_a);
        const T eh = ET0[0], el = eta_prev;
        T conv = uz * (UZp[0] - UZm[0]);
        {
          const T sx = (UX0[0] + UXm[0]) + (UX0[1] + UXm[1]);
          T tr = sx * (UZ0[1] - UZ0[-1]);
          if (DIM == 3) {
            const T sy = (UY0[0] + UYm[0]) + (UY0[EY] + UYm[EY]);
            tr += sy * (UZ0[EY] - UZ0[-EY]);
          }
          conv += T(0.25) * tr;
        }
        T V;
        if (AXI) {
          // (1/r) d_r(r 2 eta d_r u_r) - 2 eta u_r / r^2 at face radius R_k
          const T inv_R = T(1) / Rk;
          V = (rk * T(2) * eh * (UZp[0] - uz) - (rk - T(1)) * T(2) * el * (uz - UZm[0])) * inv_R;
          V -= (el + eh) * uz * inv_R * inv_R;
        } else {
          V = T(2) * (eh * (UZp[0] - uz) - el * (uz - UZm[0]));
        }
        T Vt = XZm[1] - XZm[0];  // shear edge fluxes between planes k-1 and k
        if (DIM == 3) Vt += YZm[EY] - YZm[0];
        const T Vb = BULK ? eh * DV[0] - el * dv_prev : T(0);
        V += T(0.25) * Vt + Vb;
        T G;
        if (!PAVG) {
          G = P0[0] - Pm[0];
        } else if (DIM == 2) {
          G = (T(4) * (P0[0] - Pm[0]) + ((P0[1] - Pm[1]) + (P0[-1] - Pm[-1]))) * T(1.0 / 6.0);
        } else {
          auto row = [&](int o) {
            return T(4) * (P0[o] - Pm[o]) + ((P0[o + 1] - Pm[o + 1]) + (P0[o - 1] - Pm[o - 1]));
          };
          G = (T(4) * row(0) + (row(EY) + row(-EY))) * T(1.0 / 36.0);
        }
        const T S = c.hsig * (phc + phl) * (MU[0] - mu_prev);
        const T B = (rho_f - c.rho_ref) * c.g[2];
        LuZ = fma(T(-0.5), conv, (-G + V + S + B) * recip(rho_f));
      }

      // ---- Shu-Osher combination of the stage (increment form) ----
      const bool bX = (i == 0 && g.bc[0] != BC_PERIODIC);
      const bool bY = (DIM == 3) && (j == 0 && g.bc[2] != BC_PERIODIC);
      T q[4] = {P0[0], UX0[0], (DIM == 3) ? UY0[0] : T(0), UZ0[0]};
      T L[4] = {Lp, LuX, LuY, LuZ};
      T out[4];
      T old[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        if (DIM == 2 && f == 2) continue;
        if (STAGE == 1) {
          out[f] = fma(dt, L[f], q[f]);
        } else {
          old[f] = qn_cur[f];
          if (STAGE == 2)
            out[f] = old[f] + T(0.25) * ((q[f] - old[f]) + dt * L[f]);
          else
            out[f] = old[f] + T(2.0 / 3.0) * ((q[f] - old[f]) + dt * L[f]);
        }
      }
      if (bX) out[1] = T(0);
      if (bY) out[2] = T(0);
      if (bZ) out[3] = T(0);
      const size_t pk = (size_t)k * ny * pitch;
      st_nt(A.dst[0] + pk, bo_own, out[0]);
      st_nt(A.dst[1] + pk, bo_own, out[1]);
      if (DIM == 3) st_nt(A.dst[2] + pk, bo_own, out[2]);
      st_nt(A.dst[3] + pk, bo_own, out[3]);
      if (MU_STORE && STAGE == 1) st_nt(A.mu + pk, bo_own, MU[0]);
      if (STAGE == 3) {
        st_nt(A.usum[0] + pk, bo_own, old[1] + out[1]);
        if (DIM == 3) st_nt(A.usum[1] + pk, bo_own, old[2] + out[2]);
        st_nt(A.usum[2] + pk, bo_own, old[3] + out[3]);
      }
    }
    mu_prev = L0[S_MU * PLANE];
    dv_prev = L0[S_DV * PLANE];
    eta_prev = L0[S_ET * PLANE + (k & 1) * PLANE];
    nu_prev = L0[S_NU * PLANE + (k & 1) * PLANE];

    gx_m = gx_0;
    gx_0 = gx_p;
    gy_m = gy_0;
    gy_0 = gy_p;
  };

  for (int k = z0; k < z1; k += 3) {
    step(std::integral_constant<int, 0>{}, k);
    if (k + 1 < z1) step(std::integral_constant<int, 1>{}, k + 1);
    if (k + 2 < z1) step(std::integral_constant<int, 2>{}, k + 2);
  }
}

// Single grid: work-group b runs the tile tile_of_block assigns to it.
template <typename T, int DIM, bool AXI, int STAGE, int TX, int TY, int SCH>
__global__ __launch_bounds__(TX* TY, FlowOcc<T>::W) void flow_stage_kernel(FlowArgs<T> A) {
  int btx, bty, btz;
  tile_of_block(A.g, btx, bty, btz);
  flow_stage_tile<T, DIM, AXI, STAGE, TX, TY, SCH>(A, btx, bty, btz);
}

// Batch of grids: work-group b runs tile tiles[b] = (case, btx, bty, btz)
// with the arguments cases[case].
template <typename T, int DIM, bool AXI, int STAGE, int TX, int TY>
__global__ __launch_bounds__(TX* TY, FlowOcc<T>::W) void flow_stage_batch_kernel(const FlowArgs<T>* __restrict__ cases,
                                                                         const int4* __restrict__ tiles) {
  const int4 t = tiles[blockIdx.x];
  const FlowArgs<T> A = cases[t.x];
  flow_stage_tile<T, DIM, AXI, STAGE, TX, TY>(A, t.y, t.z, t.w);
}

template <typename T, int DIM, bool AXI, int STAGE>
static hipError_t launch_flow_t(const FlowArgs<T>& a, int scheme, hipStream_t s) {
  constexpr int TX = FlowTile<DIM, T>::TX, TY = FlowTile<DIM, T>::TY;
  FlowArgs<T> b = a;
  b.g.nb[0] = (a.g.n[0] + TX - 1) / TX;
  b.g.nb[1] = (a.g.n[1] + TY - 1) / TY;
  b.g.nb[2] = (a.g.n[2] + a.g.zchunk - 1) / a.g.zchunk;
  const unsigned nblk = (unsigned)(b.g.nb[0] * b.g.nb[1] * b.g.nb[2]);
  const dim3 grid(nblk), block(TX * TY);
  switch (scheme) {
    case GPE_SCHEME_PAPER:
      hipLaunchKernelGGL((flow_stage_kernel<T, DIM, AXI, STAGE, TX, TY, 0>), grid, block, 0, s, b);
      break;
    case GPE_SCHEME_NO_PAVG:  // ablation variants: 3-D only
      if (DIM != 3) return hipErrorInvalidValue;
      hipLaunchKernelGGL((flow_stage_kernel<T, DIM, AXI, STAGE, TX, TY, DIM == 3 ? 1 : 0>), grid, block, 0, s, b);
      break;
    case GPE_SCHEME_NO_BULK:
      if (DIM != 3) return hipErrorInvalidValue;
      hipLaunchKernelGGL((flow_stage_kernel<T, DIM, AXI, STAGE, TX, TY, DIM == 3 ? 2 : 0>), grid, block, 0, s, b);
      break;
    case GPE_SCHEME_NO_PAVG | GPE_SCHEME_NO_BULK:
      if (DIM != 3) return hipErrorInvalidValue;
      hipLaunchKernelGGL((flow_stage_kernel<T, DIM, AXI, STAGE, TX, TY, DIM == 3 ? 3 : 0>), grid, block, 0, s, b);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int DIM, bool AXI>
static hipError_t launch_flow_g(const FlowArgs<T>& a, int stage, int scheme, hipStream_t s) {
  switch (stage) {
    case 1: return launch_flow_t<T, DIM, AXI, 1>(a, scheme, s);
    case 2: return launch_flow_t<T, DIM, AXI, 2>(a, scheme, s);
    case 3: return launch_flow_t<T, DIM, AXI, 3>(a, scheme, s);
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_flow(const FlowArgs<T>& a, int geometry, int stage, int scheme, hipStream_t s) {
  switch (geometry) {
    case 0: return launch_flow_g<T, 2, false>(a, stage, scheme, s);
    case 1: return launch_flow_g<T, 2, true>(a, stage, scheme, s);
    case 2: return launch_flow_g<T, 3, false>(a, stage, scheme, s);
  }
  return hipErrorInvalidValue;
}

template <typename T, bool AXI, int STAGE>
static hipError_t launch_flow_batch_t(const FlowArgs<T>* cases, const int4* tiles, int ntiles, hipStream_t s) {
  constexpr int TX = FlowTile<2, T>::TX, TY = FlowTile<2, T>::TY;
  hipLaunchKernelGGL((flow_stage_batch_kernel<T, 2, AXI, STAGE, TX, TY>), dim3((unsigned)ntiles), dim3(TX * TY), 0,
                     s, cases, tiles);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_flow_batch(const FlowArgs<T>* cases, const int4* tiles, int ntiles, int geometry, int stage,
                             hipStream_t s) {
  if (ntiles < 1) return hipErrorInvalidValue;
  const bool axi = geometry == 1;
  if (geometry != 0 && geometry != 1) return hipErrorInvalidValue;
  switch (stage) {
    case 1: return axi ? launch_flow_batch_t<T, true, 1>(cases, tiles, ntiles, s)
                       : launch_flow_batch_t<T, false, 1>(cases, tiles, ntiles, s);
    case 2: return axi ? launch_flow_batch_t<T, true, 2>(cases, tiles, ntiles, s)
                       : launch_flow_batch_t<T, false, 2>(cases, tiles, ntiles, s);
    case 3: return axi ? launch_flow_batch_t<T, true, 3>(cases, tiles, ntiles, s)
                       : launch_flow_batch_t<T, false, 3>(cases, tiles, ntiles, s);
  }
  return hipErrorInvalidValue;
}

template hipError_t launch_flow<float>(const FlowArgs<float>&, int, int, int, hipStream_t);
template hipError_t launch_flow<double>(const FlowArgs<double>&, int, int, int, hipStream_t);
template hipError_t launch_flow_batch<float>(const FlowArgs<float>*, const int4*, int, int, int, hipStream_t);
template hipError_t launch_flow_batch<double>(const FlowArgs<double>*, const int4*, int, int, int, hipStream_t);

}  // namespace gpe
