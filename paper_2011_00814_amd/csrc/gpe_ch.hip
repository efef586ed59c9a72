// gpe_ch.hip -- one stage of the Cahn-Hilliard sub-step (arXiv 2011.00814,
// Sec. 2 CH equation and chemical potential, Sec. 3 isotropic lattice
// stencils, TVD-RK2 / RK4 integration, space-time averaged centre velocity).
//
// Right-hand side (conservative transport of phi by the frozen centre
// velocity u_hat, mobility M, chemical potential mu(phi)):
//   L = -3 sum_i w_i e_i . (phi u_hat)(x + e_i) + 6 M sum_i w_i (mu(x + e_i) - mu(x))
// In axisymmetric geometry the flux is the isotropic divergence of r phi u_hat
// divided by r, and every Laplacian link is weighted by its mid-point radius.
//
// A work-group owns TX x TY columns and marches along Z.  For each new plane
// m = k+1 it stages phi (plane m+1) and the face velocity sums, then forms
// mu(m) and the flux vector F(m) = phi u_hat once in LDS rings; the output
// plane k reads mu and F from planes k-1, k, k+1.
#include "gpe_plane.hpp"

namespace gpe {

template <typename T, int DIM, bool AXI, int STAGE, int TX, int TY>
__global__ __launch_bounds__(TX* TY) void ch_stage_kernel(ChArgs<T> A) {
  constexpr int NT = TX * TY;
  constexpr int PX = TX + 4;                  // in-plane X range [-2, TX+1]
  constexpr int PY = (DIM == 3) ? TY + 4 : 1;
  constexpr int PLANE = PX * PY;
  constexpr int EY = (DIM == 3) ? PX : 0;
  constexpr int S_PH = 0;           // 3-slot ring: phi planes
  constexpr int S_SX = 3;           // 1 slot: X face sums of plane m
  constexpr int S_SY = 4;           // 1 slot: Y face sums of plane m
  constexpr int S_SZ = 5;           // 2-slot ring: Z face sums
  constexpr int S_MU = 7;           // 3-slot ring: mu
  constexpr int S_FX = 10, S_FY = 13, S_FZ = 16;  // 3-slot rings: flux components
  constexpr int NSLOT = 19;
  __shared__ T lds[NSLOT * PLANE];

  const Grid& g = A.g;
  const Consts<T>& c = A.c;
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const int tx = (int)threadIdx.x % TX, ty = (int)threadIdx.x / TX;
  const int x0 = (int)blockIdx.x * TX, y0 = (int)blockIdx.y * TY;
  const int z0 = (int)blockIdx.z * g.zchunk;
  const int z1 = min(z0 + g.zchunk, nz);
  const int i = x0 + tx, j = (DIM == 3) ? y0 + ty : 0;
  const bool active = i < nx && j < ny;
  const int own = ((DIM == 3) ? (ty + 2) * PX : 0) + tx + 2;

  PlaneMap<T, DIM, PX, PY, NT> pm;
  pm.init(g, x0, y0);

  const T* __restrict__ phin = A.phi_in;
  const T* __restrict__ s_x = A.usum[0];
  const T* __restrict__ s_y = A.usum[1];
  const T* __restrict__ s_z = A.usum[2];

  auto slot3 = [](int k) { return (k + 3) % 3; };
  auto slot2 = [](int k) { return (k + 4) % 2; };

  auto load_phi = [&](int k) {
    const ZMap<T> z(g, k);
    T* dst = &lds[(S_PH + slot3(k)) * PLANE];
#pragma unroll
    for (int p = 0; p < pm.NPASS; ++p) {
      const int lp = (int)threadIdx.x + p * NT;
      if (lp >= PLANE) continue;
      dst[lp] = pm.ok[p] ? phin[z.zc + pm.off_c[p]] : T(0);
    }
  };
  auto load_sz = [&](int k) {
    const ZMap<T> z(g, k);
    T* dst = &lds[(S_SZ + slot2(k)) * PLANE];
#pragma unroll
    for (int p = 0; p < pm.NPASS; ++p) {
      const int lp = (int)threadIdx.x + p * NT;
      if (lp >= PLANE) continue;
      dst[lp] = pm.ok[p] ? s_z[z.zf + pm.off_c[p]] * (pm.sg_z[p] * z.nrm) : T(0);
    }
  };
  auto load_sxy = [&](int k) {
    const ZMap<T> z(g, k);
#pragma unroll
    for (int p = 0; p < pm.NPASS; ++p) {
      const int lp = (int)threadIdx.x + p * NT;
      if (lp >= PLANE) continue;
      T vx = T(0), vy = T(0);
      if (pm.ok[p]) {
        vx = s_x[z.zc + pm.off_x[p]] * (pm.sg_x[p] * z.tan);
        if (DIM == 3) vy = s_y[z.zc + pm.off_y[p]] * (pm.sg_y[p] * z.tan);
      }
      lds[S_SX * PLANE + lp] = vx;
      if (DIM == 3) lds[S_SY * PLANE + lp] = vy;
    }
  };

  // mu(m) and F(m) = [r] phi u_hat on the region [-1, T] of plane m
  auto derive = [&](int m) {
    const T* F0 = &lds[(S_PH + slot3(m)) * PLANE];
    const T* Fm = &lds[(S_PH + slot3(m - 1)) * PLANE];
    const T* Fp = &lds[(S_PH + slot3(m + 1)) * PLANE];
    const T* SX = &lds[S_SX * PLANE];
    const T* SY = &lds[S_SY * PLANE];
    const T* SZ0 = &lds[(S_SZ + slot2(m)) * PLANE];
    const T* SZ1 = &lds[(S_SZ + slot2(m + 1)) * PLANE];
    T* MU = &lds[(S_MU + slot3(m)) * PLANE];
    T* FX = &lds[(S_FX + slot3(m)) * PLANE];
    T* FY = &lds[(S_FY + slot3(m)) * PLANE];
    T* FZ = &lds[(S_FZ + slot3(m)) * PLANE];
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
    constexpr int EXN = TX + 2;
    constexpr int EN = (DIM == 3) ? (TX + 2) * (TY + 2) : TX + 2;
    for (int e = (int)threadIdx.x; e < EN; e += NT) {
      const int ex = e % EXN, ey = e / EXN;
      const int q = ((DIM == 3) ? (ey + 1) * PX : 0) + ex + 1;
      const T f = F0[q];
      T lap;
      if (DIM == 2) {
        const T s1 = (F0[q + 1] - f) + (F0[q - 1] - f) + rp * (Fp[q] - f) + rm * (Fm[q] - f);
        const T s2 = rp * ((Fp[q + 1] - f) + (Fp[q - 1] - f)) + rm * ((Fm[q + 1] - f) + (Fm[q - 1] - f));
        lap = c.w1 * s1 + c.w2 * s2;
      } else {
        const T s1 = ((F0[q + 1] - f) + (F0[q - 1] - f)) + ((F0[q + EY] - f) + (F0[q - EY] - f)) +
                     ((Fp[q] - f) + (Fm[q] - f));
        lap = c.w1 * s1;
        if (c.w2 != T(0)) {
          const T s2 = ((F0[q + 1 + EY] - f) + (F0[q + 1 - EY] - f) + (F0[q - 1 + EY] - f) +
                        (F0[q - 1 - EY] - f)) +
                       ((Fp[q + 1] - f) + (Fp[q - 1] - f) + (Fp[q + EY] - f) + (Fp[q - EY] - f)) +
                       ((Fm[q + 1] - f) + (Fm[q - 1] - f) + (Fm[q + EY] - f) + (Fm[q - EY] - f));
          lap += c.w2 * s2;
        }
        if (c.w3 != T(0)) {
          const T s3 = ((Fp[q + 1 + EY] - f) + (Fp[q + 1 - EY] - f) + (Fp[q - 1 + EY] - f) +
                        (Fp[q - 1 - EY] - f)) +
                       ((Fm[q + 1 + EY] - f) + (Fm[q + 1 - EY] - f) + (Fm[q - 1 + EY] - f) +
                        (Fm[q - 1 - EY] - f));
          lap += c.w3 * s3;
        }
      }
      MU[q] = c.a4 * f * (f * f - T(1)) - c.kappa6 * lap;
      const T pr = AXI ? f * rnode : f;
      FX[q] = pr * (T(0.25) * (SX[q] + SX[q + 1]));
      if (DIM == 3) FY[q] = pr * (T(0.25) * (SY[q] + SY[q + EY]));
      FZ[q] = pr * (T(0.25) * (SZ0[q] + SZ1[q]));
    }
  };

  // -------- warm-up -------------------------------------------------------
  load_phi(z0 - 2);
  load_phi(z0 - 1);
  load_sz(z0 - 1);
  // iterations k = z0-2, z0-1 only stage and derive planes z0-1, z0
  for (int k = z0 - 2; k < z1; ++k) {
    load_phi(k + 2);
    load_sxy(k + 1);
    load_sz(k + 2);
    __syncthreads();
    derive(k + 1);
    __syncthreads();
    if (k >= z0 && active) {
      const int sm = slot3(k - 1), s0 = slot3(k), s1 = slot3(k + 1);
      const T* M0 = &lds[(S_MU + s0) * PLANE + own];
      const T* Mm = &lds[(S_MU + sm) * PLANE + own];
      const T* Mp = &lds[(S_MU + s1) * PLANE + own];
      const T* X0 = &lds[(S_FX + s0) * PLANE + own];
      const T* Xm = &lds[(S_FX + sm) * PLANE + own];
      const T* Xp = &lds[(S_FX + s1) * PLANE + own];
      const T* Y0 = &lds[(S_FY + s0) * PLANE + own];
      const T* Ym = &lds[(S_FY + sm) * PLANE + own];
      const T* Yp = &lds[(S_FY + s1) * PLANE + own];
      const T* Z0 = &lds[(S_FZ + s0) * PLANE + own];
      const T* Zm = &lds[(S_FZ + sm) * PLANE + own];
      const T* Zp = &lds[(S_FZ + s1) * PLANE + own];
      T rp = T(1), rm = T(1), inv_r = T(1);
      if (AXI) {
        const T rk = T(k) + T(0.5);
        rp = (rk + T(0.5)) / rk;
        rm = (rk - T(0.5)) / rk;
        inv_r = T(1) / rk;
      }
      const T mc = M0[0];
      T lap, flux;
      if (DIM == 2) {
        const T s1 = (M0[1] - mc) + (M0[-1] - mc) + rp * (Mp[0] - mc) + rm * (Mm[0] - mc);
        const T s2 = rp * ((Mp[1] - mc) + (Mp[-1] - mc)) + rm * ((Mm[1] - mc) + (Mm[-1] - mc));
        lap = c.w1 * s1 + c.w2 * s2;
        // D2Q9 in the (X, Z) plane: axis links and the four diagonals
        const T f1 = (X0[1] - X0[-1]) + (Zp[0] - Zm[0]);
        const T f2 = ((Xp[1] - Xp[-1]) + (Xm[1] - Xm[-1])) + ((Zp[1] + Zp[-1]) - (Zm[1] + Zm[-1]));
        flux = (c.w1 * f1 + c.w2 * f2) * inv_r;
      } else {
        const T s1 = ((M0[1] - mc) + (M0[-1] - mc)) + ((M0[EY] - mc) + (M0[-EY] - mc)) +
                     ((Mp[0] - mc) + (Mm[0] - mc));
        lap = c.w1 * s1;
        flux = c.w1 * ((X0[1] - X0[-1]) + (Y0[EY] - Y0[-EY]) + (Zp[0] - Zm[0]));
        if (c.w2 != T(0)) {
          const T s2 = ((M0[1 + EY] - mc) + (M0[1 - EY] - mc) + (M0[-1 + EY] - mc) + (M0[-1 - EY] - mc)) +
                       ((Mp[1] - mc) + (Mp[-1] - mc) + (Mp[EY] - mc) + (Mp[-EY] - mc)) +
                       ((Mm[1] - mc) + (Mm[-1] - mc) + (Mm[EY] - mc) + (Mm[-EY] - mc));
          lap += c.w2 * s2;
          // edges: XY in plane k, XZ and YZ in planes k +- 1
          const T exy = ((X0[1 + EY] + X0[1 - EY]) - (X0[-1 + EY] + X0[-1 - EY])) +
                        ((Y0[1 + EY] + Y0[-1 + EY]) - (Y0[1 - EY] + Y0[-1 - EY]));
          const T exz = ((Xp[1] - Xp[-1]) + (Xm[1] - Xm[-1])) + ((Zp[1] + Zp[-1]) - (Zm[1] + Zm[-1]));
          const T eyz = ((Yp[EY] - Yp[-EY]) + (Ym[EY] - Ym[-EY])) + ((Zp[EY] + Zp[-EY]) - (Zm[EY] + Zm[-EY]));
          flux += c.w2 * (exy + (exz + eyz));
        }
        if (c.w3 != T(0)) {
          const T s3 = ((Mp[1 + EY] - mc) + (Mp[1 - EY] - mc) + (Mp[-1 + EY] - mc) + (Mp[-1 - EY] - mc)) +
                       ((Mm[1 + EY] - mc) + (Mm[1 - EY] - mc) + (Mm[-1 + EY] - mc) + (Mm[-1 - EY] - mc));
          lap += c.w3 * s3;
          // corners (sx, sy, sz): sx F_X + sy F_Y + sz F_Z at planes k +- 1
          auto corner = [&](const T* X, const T* Y) {
            return ((X[1 + EY] + X[1 - EY]) - (X[-1 + EY] + X[-1 - EY])) +
                   ((Y[1 + EY] + Y[-1 + EY]) - (Y[1 - EY] + Y[-1 - EY]));
          };
          const T zs = ((Zp[1 + EY] + Zp[1 - EY]) + (Zp[-1 + EY] + Zp[-1 - EY])) -
                       ((Zm[1 + EY] + Zm[1 - EY]) + (Zm[-1 + EY] + Zm[-1 - EY]));
          flux += c.w3 * ((corner(Xp, Yp) + corner(Xm, Ym)) + zs);
        }
      }
      const T L = T(-3) * flux + T(6) * c.mob * lap;
      const size_t ci = ((size_t)k * ny + j) * nx + i;
      const T dt = c.dt;
      const T phc = lds[(S_PH + s0) * PLANE + own];
      if (STAGE == CH_RK2_1) {
        A.out[ci] = phc + dt * L;
      } else if (STAGE == CH_RK2_2) {
        const T ps = A.phis[ci];
        A.out[ci] = ps + T(0.5) * ((phc - ps) + dt * L);
      } else if (STAGE == CH_RK4_1) {
        const T kk = dt * L;
        A.out[ci] = phc + T(0.5) * kk;
        A.acc[ci] = phc + kk * T(1.0 / 6.0);
      } else if (STAGE == CH_RK4_2) {
        const T kk = dt * L;
        A.out[ci] = A.phis[ci] + T(0.5) * kk;
        A.acc[ci] = A.acc[ci] + kk * T(1.0 / 3.0);
      } else if (STAGE == CH_RK4_3) {
        const T kk = dt * L;
        A.out[ci] = A.phis[ci] + kk;
        A.acc[ci] = A.acc[ci] + kk * T(1.0 / 3.0);
      } else {
        const T kk = dt * L;
        A.out[ci] = A.acc[ci] + kk * T(1.0 / 6.0);
      }
    }
    __syncthreads();
  }
}

template <typename T, int DIM, bool AXI, int STAGE>
static hipError_t launch_ch_t(const ChArgs<T>& a, hipStream_t s) {
  constexpr int TX = ChTile<DIM>::TX, TY = ChTile<DIM>::TY;
  dim3 grid((a.g.n[0] + TX - 1) / TX, (a.g.n[1] + TY - 1) / TY,
            (a.g.n[2] + a.g.zchunk - 1) / a.g.zchunk);
  hipLaunchKernelGGL((ch_stage_kernel<T, DIM, AXI, STAGE, TX, TY>), grid, dim3(TX * TY), 0, s, a);
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

template hipError_t launch_ch<float>(const ChArgs<float>&, int, int, hipStream_t);
template hipError_t launch_ch<double>(const ChArgs<double>&, int, int, hipStream_t);

}  // namespace gpe
