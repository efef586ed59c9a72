// gpe_ch.hip -- one stage of the Cahn-Hilliard sub-step (arXiv 2011.00814,
// Sec. 2 CH equation and chemical potential, Sec. 3 isotropic lattice
// stencils, TVD-RK2 / RK4 integration, space-time averaged centre velocity).
//
// Right-hand side (transport of phi by the frozen centre velocity u_hat,
// mobility M, chemical potential mu(phi)), conservative form (ADV = false):
//   L = -3 sum_i w_i e_i . (phi u_hat)(x + e_i) + 6 M sum_i w_i (mu(x + e_i) - mu(x))
// or advective form (ADV = true, the CH equation as printed):
//   L = -3 u_hat(x) . sum_i w_i e_i phi(x + e_i) + 6 M sum_i w_i (mu(x + e_i) - mu(x))
// In axisymmetric geometry the conservative flux is the isotropic divergence
// of r phi u_hat divided by r (the advective gradient carries no radius), and
// every Laplacian link is weighted by its mid-point radius.
//
// A work-group owns TX x TY columns and marches along Z.  For each new plane
// m = k+1 it stages phi (plane m+1) and the face velocity sums, then forms
// mu(m) and the flux vector F(m) = phi u_hat once in LDS rings; the output
// plane k reads mu and F from planes k-1, k, k+1.  In the advective form the
// F_X ring holds a copy of phi(m) instead (the phi ring has already dropped
// plane k-1 when plane k is written) and each thread keeps the centre
// velocity of its own cell in registers from derive(k) to output(k).
#include <type_traits>

#include "gpe_plane.hpp"

namespace gpe {

// Occupancy target: 6 waves per SIMD in FP32 (<= 80 VGPRs; three
// work-groups of 512 threads per CU fit the LDS footprint below); FP64 is
// LDS-limited to 2.
template <typename T>
struct ChOcc { static constexpr int W = sizeof(T) == 4 ? 6 : 2; };

// One work-group tile (btx, bty) x Z chunk btz of the grid described by A.
template <typename T, int DIM, bool AXI, int STAGE, int TX, int TY, bool ADV>
__device__ __forceinline__ void ch_stage_tile(const ChArgs<T>& A, int btx, int bty, int btz) {
  constexpr int NT = TX * TY;
  constexpr int PX = TX + 4;                  // in-plane X range [-2, TX+1]
  constexpr int PY = (DIM == 3) ? TY + 4 : 1;
  constexpr int PLANE = PX * PY;
  constexpr int EY = (DIM == 3) ? PX : 0;
  // mu and the flux components live on [-1, T] only: a tighter plane
  constexpr int QX = TX + 2;
  constexpr int QY = (DIM == 3) ? TY + 2 : 1;
  constexpr int QPLANE = QX * QY;
  constexpr int QEY = (DIM == 3) ? QX : 0;
  // 3-slot rings (slot of plane m = (m - z0) mod 3) of phi and the Z face
  // sums, single slots of the X / Y face sums of one plane (halo'd plane);
  // 3-slot rings of mu and the flux components (tight plane)
  constexpr int S_PH = 0, S_SZ = 3, S_SX = 6, S_SY = 7, NSLOT = 8;
  constexpr int S_MU = 0, S_FX = 3, S_FY = 6, S_FZ = 9, NQSLOT = 12;
  __shared__ T lds[NSLOT * PLANE];
  __shared__ T ldq[NQSLOT * QPLANE];

  const Grid& g = A.g;
  const Consts<T>& c = A.c;
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2], pitch = g.pitch;
  const int tx = (int)threadIdx.x % TX, ty = (int)threadIdx.x / TX;
  const int x0 = btx * TX, y0 = bty * TY;
  const int z0 = btz * g.zchunk;
  __builtin_assume(z0 >= 0);  // lets the plane-index checks of the staging fold
  const int z1 = min(z0 + g.zchunk, nz);
  const int i = x0 + tx, j = (DIM == 3) ? y0 + ty : 0;
  const bool active = i < nx && j < ny;
  const int ij = j * pitch + i;  // in-plane offset of the own column
  const int own = ((DIM == 3) ? (ty + 2) * PX : 0) + tx + 2;
  const T* const L0 = lds + own;
  const T* const Q0 = ldq + ((DIM == 3) ? (ty + 1) * QX : 0) + tx + 1;

  PlaneMap<T, DIM, PX, PY, NT> pm;
  pm.init(g, x0, y0);

  // Staging of the planes an iteration needs (phi of plane k+2, the X/Y face
  // sums of plane k+1, the Z face sums of plane k+2) is software-pipelined:
  // fetch() issues the global loads into registers one iteration ahead,
  // commit() applies the ghost-rule signs and writes them to LDS.  No
  // arithmetic touches a loaded value before commit(), so the loads stay in
  // flight while the current plane is processed.  A plane index below -2
  // marks "nothing to stage" (only in the warm-up, where the indices are
  // constants).  Every lane issues every load, so no branch separates the
  // loads from the waits for them: a position outside the mapped halo
  // (never read) loads the plane's first element instead, and the face sums
  // are loaded on the outermost row too (never read there either).
  constexpr int NP = PlaneMap<T, DIM, PX, PY, NT>::NPASS;
  struct Staged {  // one iteration's loaded values, per load pass
    T f[NP], x[NP], y[NP], z[NP];
  };
  Staged R;  // the values in flight in the main loop
  // byte offsets of every load pass within a plane (loop invariant): the
  // cell value and the X / Y face values of the position
  uint32_t bo_c[NP], bo_x[NP], bo_y[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const auto q = pm.pos(g, p);
    const bool ok = pm.ok[p];
    bo_c[p] = (uint32_t)(ok ? q.oc : 0) * (uint32_t)sizeof(T);
    bo_x[p] = (uint32_t)(ok ? q.ox : 0) * (uint32_t)sizeof(T);
    bo_y[p] = (uint32_t)(ok ? q.oy : 0) * (uint32_t)sizeof(T);
  }
  auto fetch = [&](int kf, int kxy, int kz, Staged& r) {
    const ZMap<T> zf(g, kf), zxy(g, kxy), zz(g, kz);
    const T* __restrict__ bf = A.phi_in + zf.zc;
    const T* __restrict__ bx = A.usum[0] + zxy.zc;
    const T* __restrict__ by = A.usum[1] + zxy.zc;
    const T* __restrict__ bz = A.usum[2] + zz.zf;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      refresh(bo_c[p]);
      refresh(bo_x[p]);
      if (DIM == 3) refresh(bo_y[p]);
      r.f[p] = (kf >= -2) ? at_b(bf, bo_c[p]) : T(0);
      r.x[p] = (kxy >= -2) ? at_b(bx, bo_x[p]) : T(0);
      r.y[p] = (DIM == 3 && kxy >= -2) ? at_b(by, bo_y[p]) : T(0);
      r.z[p] = (kz >= -2) ? at_b(bz, bo_c[p]) : T(0);
    }
  };
  auto commit = [&](int kxy, int kz, int sf, int sz, bool do_f, bool do_xy, bool do_z, const Staged& r) {
    const ZMap<T> zxy(g, kxy), zz(g, kz);
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const int lp = (int)threadIdx.x + p * NT;
      if (lp >= PLANE) continue;
      const auto q = pm.pos(g, p);  // signs (all +1 inside an interior tile)
      if (do_f) lds[(S_PH + sf) * PLANE + lp] = r.f[p];
      if (do_xy) {
        lds[S_SX * PLANE + lp] = r.x[p] * (q.sx * zxy.tan);
        if (DIM == 3) lds[S_SY * PLANE + lp] = r.y[p] * (q.sy * zxy.tan);
      }
      if (do_z) lds[(S_SZ + sz) * PLANE + lp] = r.z[p] * (q.sz * zz.nrm);
    }
  };

  // mu(m) and F(m) = [r] phi u_hat on the region [-1, T] of plane m whose
  // ring slot is SC (planes m-1, m+1 in SM, SP)
  auto derive = [&](int m, auto sc) {
    constexpr int SC = decltype(sc)::value;
    constexpr int SM = (SC + 2) % 3, SP = (SC + 1) % 3;
    T rp = T(1), rm = T(1), rnode = T(1);
    if (AXI) {
      // A ghost plane beyond the axis or the outer wall mirrors an in-domain
      // row: use that row's radius, with the up/down link weights exchanged,
      // so that mu on the ghost plane is the mirror image of mu on the row.
      const ZMap<T> z(g, m);
      const T rk = z.r;
      const T up = (rk + T(0.5)) / rk, dn = (rk - T(0.5)) / rk;
      const bool mirrored = m < 0 || m >= nz;
      rp = mirrored ? dn : up;
      rm = mirrored ? up : dn;
      rnode = rk;
    }
    constexpr int EN = (DIM == 3) ? (TX + 2) * (TY + 2) : TX + 2;
    for (int e = (int)threadIdx.x; e < EN; e += NT) {
      int ex, ey;
      region_pos<TX + 2, (DIM == 3) ? TY + 2 : 1>(e, ex, ey);
      const int q = ((DIM == 3) ? (ey + 1) * PX : 0) + ex + 1;
      const T* b = lds + q;
      T* bq = ldq + ey * QX + ex;
      const T* F0 = b + (S_PH + SC) * PLANE;
      const T* Fm = b + (S_PH + SM) * PLANE;
      const T* Fp = b + (S_PH + SP) * PLANE;
      const T f = F0[0];
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
      bq[(S_MU + SC) * QPLANE] = c.a4 * f * (f * f - T(1)) - c.kappa6 * lap;
      if (ADV) {
        bq[(S_FX + SC) * QPLANE] = f;
        continue;
      }
      // centre velocity = 1/4 of the sums over its two faces; the factor 1/4
      // is applied in the flux divergence
      const T pr = AXI ? f * rnode : f;
      const T* SX = b + S_SX * PLANE;
      const T* SY = b + S_SY * PLANE;
      bq[(S_FX + SC) * QPLANE] = pr * (SX[0] + SX[1]);
      if (DIM == 3) bq[(S_FY + SC) * QPLANE] = pr * (SY[0] + SY[EY]);
      bq[(S_FZ + SC) * QPLANE] = pr * (b[(S_SZ + SC) * PLANE] + b[(S_SZ + SP) * PLANE]);
    }
  };

  // pointwise stage inputs (phi* and the RK4 running sum) at the thread's
  // own cell, loaded one plane ahead of their use
  constexpr bool NEED_PHIS = STAGE == CH_RK2_2 || STAGE == CH_RK4_2 || STAGE == CH_RK4_3 || STAGE == CH_RK4_4;
  constexpr bool NEED_ACC = STAGE == CH_RK2_2 || STAGE == CH_RK4_2 || STAGE == CH_RK4_3 || STAGE == CH_RK4_4;
  T phis_cur = T(0), acc_cur = T(0), phis_next = T(0), acc_next = T(0);
  // advective form: 4 u_hat of the own cell (sums over its two faces) of the
  // plane being written and of the next one
  T uc_cur[3] = {T(0), T(0), T(0)}, uc_next[3] = {T(0), T(0), T(0)};
  // (unconditional: outside the chunk, or in an inactive lane, it loads a
  // value of the chunk that is never used)
  uint32_t bo_own = (uint32_t)(active ? ij : 0) * (uint32_t)sizeof(T);
  auto fetch_pt = [&](int k, T& ps, T& ac) {
    const size_t po = (size_t)min(max(k, z0), z1 - 1) * ny * pitch;
    refresh(bo_own);
    if (NEED_PHIS) ps = ld_nt(A.phis + po, bo_own);
    if (NEED_ACC) ac = ld_nt(A.acc + po, bo_own);
  };

  // FP64: the values of plane k are stored one iteration later, right after
  // the next plane's commit and before its loads; a store issued after the
  // loads sits behind a branch (warm-up iterations and ragged lanes store
  // nothing), and the compiler would then wait for it together with the
  // loads at the next commit (measured: the FP64 stages 4-6 % faster, FP32
  // stages 0.5 % slower, so FP32 stores at once).
  constexpr bool DEFER = sizeof(T) == 8;
  T pv_out = T(0), pv_acc = T(0);
  constexpr bool WRITES_ACC = STAGE == CH_RK2_1 || STAGE == CH_RK4_1 || STAGE == CH_RK4_2 || STAGE == CH_RK4_3;
  auto store = [&](int k) {
    if (k >= z0 && active) {
      const size_t po = (size_t)k * ny * pitch;
      st_nt(A.out + po, bo_own, pv_out);
      if (WRITES_ACC) st_nt(A.acc + po, bo_own, pv_acc);
    }
  };

  // Corner sums of one plane at the own column, for the corner links
  // (+-1, +-1, +-1) of the 3-D lattices: q[0] the sum of mu over the four
  // in-plane diagonal neighbours; conservative form q[1] = sum of
  // sx F_X + sy F_Y and q[2] = sum of F_Z over them; advective form q[1..3]
  // = the sums of sx phi, sy phi and phi.  The output of plane k takes them
  // for planes k + 1 and k - 1; the sums of plane m are formed once, right
  // after plane m is derived, and carried in registers until the output of
  // plane m + 1 (instead of reading the same 16 LDS words again there).
  auto corners = [&](auto sm, T* q) {
    constexpr int SC = decltype(sm)::value;
    const T* M = Q0 + (S_MU + SC) * QPLANE;
    const T* X = Q0 + (S_FX + SC) * QPLANE;
    q[0] = (M[1 + QEY] + M[1 - QEY]) + (M[-1 + QEY] + M[-1 - QEY]);
    if (!ADV) {
      const T* Y = Q0 + (S_FY + SC) * QPLANE;
      const T* Z = Q0 + (S_FZ + SC) * QPLANE;
      q[1] = ((X[1 + QEY] + X[1 - QEY]) - (X[-1 + QEY] + X[-1 - QEY])) +
             ((Y[1 + QEY] + Y[-1 + QEY]) - (Y[1 - QEY] + Y[-1 - QEY]));
      q[2] = (Z[1 + QEY] + Z[1 - QEY]) + (Z[-1 + QEY] + Z[-1 - QEY]);
    } else {
      q[1] = (X[1 + QEY] + X[1 - QEY]) - (X[-1 + QEY] + X[-1 - QEY]);
      q[2] = (X[1 + QEY] + X[-1 + QEY]) - (X[1 - QEY] + X[-1 - QEY]);
      q[3] = (X[1 + QEY] + X[1 - QEY]) + (X[-1 + QEY] + X[-1 - QEY]);
    }
  };
  constexpr int NC = ADV ? 4 : 3;
  T cq_m[4] = {T(0), T(0), T(0), T(0)};  // planes k - 1, k, k + 1
  T cq_0[4] = {T(0), T(0), T(0), T(0)};
  T cq_p[4] = {T(0), T(0), T(0), T(0)};

  // output at plane k whose ring slot is S0 (planes k-1, k+1 in SM, SP);
  // phc = phi(k) at the own cell
  auto output = [&](int k, auto s0, T phc, T ps, T ac, T ucx, T ucy, T ucz, const T* cp, const T* cm) {
    constexpr int S0 = decltype(s0)::value;
    constexpr int SM = (S0 + 2) % 3, SP = (S0 + 1) % 3;
    const T* M0 = Q0 + (S_MU + S0) * QPLANE;
    const T* Mm = Q0 + (S_MU + SM) * QPLANE;
    const T* Mp = Q0 + (S_MU + SP) * QPLANE;
    const T* X0 = Q0 + (S_FX + S0) * QPLANE;
    const T* Xm = Q0 + (S_FX + SM) * QPLANE;
    const T* Xp = Q0 + (S_FX + SP) * QPLANE;
    const T* Y0 = Q0 + (S_FY + S0) * QPLANE;
    const T* Ym = Q0 + (S_FY + SM) * QPLANE;
    const T* Yp = Q0 + (S_FY + SP) * QPLANE;
    const T* Zm = Q0 + (S_FZ + SM) * QPLANE;
    const T* Zp = Q0 + (S_FZ + SP) * QPLANE;
    T rp = T(1), rm = T(1), inv_r = T(1);
    if (AXI) {
      const T rk = T(k) + T(0.5);
      inv_r = T(1) / rk;
      rp = (rk + T(0.5)) * inv_r;
      rm = (rk - T(0.5)) * inv_r;
    }
    const T mc = M0[0];
    T lap, flux;
    if (DIM == 2) {
      const T s1 = ((M0[1] - mc) + (M0[-1] - mc)) + (rp * (Mp[0] - mc) + rm * (Mm[0] - mc));
      const T s2 = rp * ((Mp[1] - mc) + (Mp[-1] - mc)) + rm * ((Mm[1] - mc) + (Mm[-1] - mc));
      lap = c.w1 * s1 + c.w2 * s2;
      if (!ADV) {
        // D2Q9 in the (X, Z) plane: axis links and the four diagonals
        const T f1 = (X0[1] - X0[-1]) + (Zp[0] - Zm[0]);
        const T f2 = ((Xp[1] - Xp[-1]) + (Xm[1] - Xm[-1])) + ((Zp[1] + Zp[-1]) - (Zm[1] + Zm[-1]));
        flux = (c.w1 * f1 + c.w2 * f2) * inv_r;
      } else {
        // isotropic gradient of phi (held in the F_X ring) along X and Z
        const T gx = c.w1 * (X0[1] - X0[-1]) + c.w2 * ((Xp[1] - Xp[-1]) + (Xm[1] - Xm[-1]));
        const T gz = c.w1 * (Xp[0] - Xm[0]) + c.w2 * ((Xp[1] + Xp[-1]) - (Xm[1] + Xm[-1]));
        flux = ucx * gx + ucz * gz;
      }
    } else {
      // Laplacian of mu summed first: mu has no offset in the bulk (it
      // vanishes there), so the neighbour sums lose nothing against the
      // differences, at half the instructions
      const T s1 = ((M0[1] + M0[-1]) + (M0[QEY] + M0[-QEY])) + (Mp[0] + Mm[0]);
      lap = fma(T(-6) * c.w1, mc, c.w1 * s1);
      // advective form: isotropic gradient of phi, held in the F_X ring
      T gx = T(0), gy = T(0), gz = T(0);
      if (!ADV) {
        flux = c.w1 * ((X0[1] - X0[-1]) + (Y0[QEY] - Y0[-QEY]) + (Zp[0] - Zm[0]));
      } else {
        gx = c.w1 * (X0[1] - X0[-1]);
        gy = c.w1 * (X0[QEY] - X0[-QEY]);
        gz = c.w1 * (Xp[0] - Xm[0]);
      }
      if (c.w2 != T(0)) {
        const T s2 = ((M0[1 + QEY] + M0[1 - QEY]) + (M0[-1 + QEY] + M0[-1 - QEY])) +
                     ((Mp[1] + Mp[-1]) + (Mp[QEY] + Mp[-QEY])) + ((Mm[1] + Mm[-1]) + (Mm[QEY] + Mm[-QEY]));
        lap += c.w2 * fma(T(-12), mc, s2);
        if (!ADV) {
          // edges: XY in plane k, XZ and YZ in planes k +- 1
          const T exy = ((X0[1 + QEY] + X0[1 - QEY]) - (X0[-1 + QEY] + X0[-1 - QEY])) +
                        ((Y0[1 + QEY] + Y0[-1 + QEY]) - (Y0[1 - QEY] + Y0[-1 - QEY]));
          const T exz = ((Xp[1] - Xp[-1]) + (Xm[1] - Xm[-1])) + ((Zp[1] + Zp[-1]) - (Zm[1] + Zm[-1]));
          const T eyz = ((Yp[QEY] - Yp[-QEY]) + (Ym[QEY] - Ym[-QEY])) + ((Zp[QEY] + Zp[-QEY]) - (Zm[QEY] + Zm[-QEY]));
          flux += c.w2 * (exy + (exz + eyz));
        } else {
          // edge links: XY in plane k, XZ / YZ in planes k +- 1
          const T* P0 = X0;
          const T* Pp = Xp;
          const T* Pm = Xm;
          gx += c.w2 * (((P0[1 + QEY] + P0[1 - QEY]) - (P0[-1 + QEY] + P0[-1 - QEY])) +
                        ((Pp[1] - Pp[-1]) + (Pm[1] - Pm[-1])));
          gy += c.w2 * (((P0[1 + QEY] + P0[-1 + QEY]) - (P0[1 - QEY] + P0[-1 - QEY])) +
                        ((Pp[QEY] - Pp[-QEY]) + (Pm[QEY] - Pm[-QEY])));
          gz += c.w2 * (((Pp[1] + Pp[-1]) + (Pp[QEY] + Pp[-QEY])) - ((Pm[1] + Pm[-1]) + (Pm[QEY] + Pm[-QEY])));
        }
      }
      if (c.w3 != T(0)) {
        // corner links (+-1, +-1, +-1): the per-plane corner sums of planes
        // k + 1 (cp) and k - 1 (cm), formed by corners()
        lap += c.w3 * fma(T(-8), mc, cp[0] + cm[0]);
        if (!ADV) {
          flux += c.w3 * ((cp[1] + cm[1]) + (cp[2] - cm[2]));
        } else {
          gx += c.w3 * (cp[1] + cm[1]);
          gy += c.w3 * (cp[2] + cm[2]);
          gz += c.w3 * (cp[3] - cm[3]);
        }
      }
      if (ADV) flux = (ucx * gx + ucy * gy) + ucz * gz;
    }
    // L = -3 sum_i w_i e_i . F(x + e_i) + 6 M sum_i w_i (mu_i - mu); the
    // stored fluxes carry 4x the centre velocity
    const T L = T(-0.75) * flux + T(6) * c.mob * lap;
    T& out = pv_out;
    T& acc = pv_acc;
    const T dt = c.dt;
    if (STAGE == CH_RK2_1) {
      // TVD-RK2 as phi* + (a + b)/2 with a = dt L kept in the running-sum
      // buffer (not recovered as (phi* + a) - phi*, which near phi = +-1
      // drops the part of a below half an ulp)
      const T kk = dt * L;
      out = phc + kk;
      acc = kk;
    } else if (STAGE == CH_RK2_2) {
      out = ps + T(0.5) * (ac + dt * L);
    } else if (STAGE == CH_RK4_1) {
      // classic RK4 with increments a, b, c, d = dt L; the running sum holds
      // the increments only, a + 2b + 2c + d, so phi* is rounded together
      // with the whole step's increment once (near phi = +-1 a small
      // increment would otherwise be rounded away at every stage)
      const T kk = dt * L;
      out = fma(T(0.5), kk, phc);
      acc = kk;
    } else if (STAGE == CH_RK4_2) {
      const T kk = dt * L;
      out = fma(T(0.5), kk, ps);
      acc = fma(T(2), kk, ac);
    } else if (STAGE == CH_RK4_3) {
      const T kk = dt * L;
      out = ps + kk;
      acc = fma(T(2), kk, ac);
    } else {
      const T kk = dt * L;
      out = ps + (ac + kk) / T(6);
    }
    if (!DEFER) store(k);
  };

  // one iteration: stage phi(k+2), the X/Y sums of plane k+1 and the Z sums
  // of plane k+2, derive mu and F of plane k+1, write plane k (k >= z0).
  // Two barriers: staged planes -> derive, derive -> output.  The next
  // iteration's staging overwrites the slots of phi(k) and the face sums,
  // whose last readers (derive, and phi(k) at the own cell, read into a
  // register) finish before the second barrier; the next derive overwrites
  // the mu / F slot of plane k-1 only after the next first barrier, which
  // every wave reaches after its output.
  auto iter = [&](int k, auto sk) {
    constexpr int SK = decltype(sk)::value;  // slot of plane k
    constexpr int S1 = (SK + 1) % 3, S2 = (SK + 2) % 3;
    wave_prio<3>();
    commit(k + 1, k + 2, S2, S2, true, true, true, R);
    if (DEFER) store(k - 1);
    fetch_pt(k + 1, phis_next, acc_next);
    {  // in flight during this plane's work; the chunk's last plane loads the
       // planes just loaded again (unused) so that the loads are unconditional
      const int d = (k + 1 < z1) ? 1 : 0;
      fetch(k + 2 + d, k + 1 + d, k + 2 + d, R);
    }
    wave_prio<0>();
    __syncthreads();
    wave_prio<1>();
    derive(k + 1, std::integral_constant<int, S1>{});
    wave_prio<0>();
    const T phc = L0[(S_PH + SK) * PLANE];
    if (ADV) {
      // face sums of plane k+1 (X / Y single slots, Z ring slots of k+1, k+2)
      uc_next[0] = L0[S_SX * PLANE] + L0[S_SX * PLANE + 1];
      uc_next[1] = (DIM == 3) ? L0[S_SY * PLANE] + L0[S_SY * PLANE + EY] : T(0);
      uc_next[2] = L0[(S_SZ + S1) * PLANE] + L0[(S_SZ + S2) * PLANE];
    }
    __syncthreads();
    const bool corner_links = DIM == 3 && c.w3 != T(0);
    if (corner_links) corners(std::integral_constant<int, S1>{}, cq_p);
    if (k >= z0 && active) output(k, sk, phc, phis_cur, acc_cur, uc_cur[0], uc_cur[1], uc_cur[2], cq_p, cq_m);
    if (corner_links) {
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        cq_m[q] = cq_0[q];
        cq_0[q] = cq_p[q];
      }
    }
    phis_cur = phis_next;
    acc_cur = acc_next;
    if (ADV) {
      uc_cur[0] = uc_next[0];
      uc_cur[1] = uc_next[1];
      uc_cur[2] = uc_next[2];
    }
  };

  // -------- warm-up: phi(z0-2), phi(z0-1) and the Z sums of plane z0-1 ----
  // (loads of both and of the first iteration issued before either commit)
  {
    Staged W0, W1;
    fetch(z0 - 2, -3, z0 - 1, W0);
    fetch(z0 - 1, -3, -3, W1);
    fetch(z0, z0 - 1, z0, R);
    commit(-3, z0 - 1, 1, 2, true, false, true, W0);
    commit(-3, -3, 2, 0, true, false, false, W1);
  }
  // iterations k = z0-2, z0-1 only stage and derive planes z0-1, z0
  for (int k = z0 - 2; k < z1; k += 3) {
    iter(k, std::integral_constant<int, 1>{});
    if (k + 1 < z1) iter(k + 1, std::integral_constant<int, 2>{});
    if (k + 2 < z1) iter(k + 2, std::integral_constant<int, 0>{});
  }
  if (DEFER) store(z1 - 1);
}

// Single grid: work-group b runs the tile tile_of_block assigns to it.
template <typename T, int DIM, bool AXI, int STAGE, int TX, int TY, bool ADV>
__global__ __launch_bounds__(TX* TY, ChOcc<T>::W) void ch_stage_kernel(ChArgs<T> A) {
  int btx, bty, btz;
  tile_of_block(A.g, btx, bty, btz);
  ch_stage_tile<T, DIM, AXI, STAGE, TX, TY, ADV>(A, btx, bty, btz);
}

// Batch of grids: work-group b runs tile tiles[b] = (case, btx, bty, btz)
// with the arguments cases[case].
template <typename T, int DIM, bool AXI, int STAGE, int TX, int TY>
__global__ __launch_bounds__(TX* TY, ChOcc<T>::W) void ch_stage_batch_kernel(const ChArgs<T>* __restrict__ cases,
                                                                         const int4* __restrict__ tiles) {
  const int4 t = tiles[blockIdx.x];
  const ChArgs<T> A = cases[t.x];
  ch_stage_tile<T, DIM, AXI, STAGE, TX, TY, false>(A, t.y, t.z, t.w);
}

template <typename T, int DIM, bool AXI, int STAGE>
static hipError_t launch_ch_t(const ChArgs<T>& a, hipStream_t s) {
  constexpr int TX = ChTile<DIM, T>::TX, TY = ChTile<DIM, T>::TY;
  ChArgs<T> b = a;
  b.g.nb[0] = (a.g.n[0] + TX - 1) / TX;
  b.g.nb[1] = (a.g.n[1] + TY - 1) / TY;
  b.g.nb[2] = (a.g.n[2] + a.g.zchunk - 1) / a.g.zchunk;
  const unsigned nblk = (unsigned)(b.g.nb[0] * b.g.nb[1] * b.g.nb[2]);
  if (a.adv)
    hipLaunchKernelGGL((ch_stage_kernel<T, DIM, AXI, STAGE, TX, TY, true>), dim3(nblk), dim3(TX * TY), 0, s, b);
  else
    hipLaunchKernelGGL((ch_stage_kernel<T, DIM, AXI, STAGE, TX, TY, false>), dim3(nblk), dim3(TX * TY), 0, s, b);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ch(const ChArgs<T>& a, int geometry, int stage, hipStream_t s) {
  if (geometry == 0) {
    if (stage == CH_RK2_1) return launch_ch_t<T, 2, false, CH_RK2_1>(a, s);
    if (stage == CH_RK2_2) return launch_ch_t<T, 2, false, CH_RK2_2>(a, s);
  } else if (geometry == 1) {
    if (stage == CH_RK2_1) return launch_ch_t<T, 2, true, CH_RK2_1>(a, s);
    if (stage == CH_RK2_2) return launch_ch_t<T, 2, true, CH_RK2_2>(a, s);
  } else if (geometry == 2) {
    switch (stage) {
      case CH_RK4_1: return launch_ch_t<T, 3, false, CH_RK4_1>(a, s);
      case CH_RK4_2: return launch_ch_t<T, 3, false, CH_RK4_2>(a, s);
      case CH_RK4_3: return launch_ch_t<T, 3, false, CH_RK4_3>(a, s);
      case CH_RK4_4: return launch_ch_t<T, 3, false, CH_RK4_4>(a, s);
    }
  }
  return hipErrorInvalidValue;
}

template <typename T, bool AXI, int STAGE>
static hipError_t launch_ch_batch_t(const ChArgs<T>* cases, const int4* tiles, int ntiles, hipStream_t s) {
  constexpr int TX = ChTile<2, T>::TX, TY = ChTile<2, T>::TY;
  hipLaunchKernelGGL((ch_stage_batch_kernel<T, 2, AXI, STAGE, TX, TY>), dim3((unsigned)ntiles), dim3(TX * TY), 0, s,
                     cases, tiles);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ch_batch(const ChArgs<T>* cases, const int4* tiles, int ntiles, int geometry, int stage,
                           hipStream_t s) {
  if (ntiles < 1) return hipErrorInvalidValue;
  if (geometry == 0) {
    if (stage == CH_RK2_1) return launch_ch_batch_t<T, false, CH_RK2_1>(cases, tiles, ntiles, s);
    if (stage == CH_RK2_2) return launch_ch_batch_t<T, false, CH_RK2_2>(cases, tiles, ntiles, s);
  } else if (geometry == 1) {
    if (stage == CH_RK2_1) return launch_ch_batch_t<T, true, CH_RK2_1>(cases, tiles, ntiles, s);
    if (stage == CH_RK2_2) return launch_ch_batch_t<T, true, CH_RK2_2>(cases, tiles, ntiles, s);
  }
  return hipErrorInvalidValue;
}

template hipError_t launch_ch<float>(const ChArgs<float>&, int, int, hipStream_t);
template hipError_t launch_ch<double>(const ChArgs<double>&, int, int, hipStream_t);
template hipError_t launch_ch_batch<float>(const ChArgs<float>*, const int4*, int, int, int, hipStream_t);
template hipError_t launch_ch_batch<double>(const ChArgs<double>*, const int4*, int, int, int, hipStream_t);

}  // namespace gpe
