// gpe_flow.hip -- one TVD-RK3 stage of the pressure and momentum equations
// (arXiv 2011.00814, Sec. 3) as a single fused kernel.
//
// Work decomposition: a work-group owns TX x TY columns of cells and marches
// along Z through ZC output planes.  Each plane of p, u_X, u_Y, u_Z and phi
// is staged once from HBM into a 3-plane LDS ring (with the in-plane halo
// and the boundary ghost rules applied while loading); eta and nu are
// derived from the frozen phi as the plane is staged; mu and div u of the
// current plane are formed once in LDS; each thread then evaluates the
// pressure RHS at its cell and the momentum RHS at the three low faces of
// its cell, applies the Shu-Osher combination of the stage and writes the
// result.  Stage 3 updates time level n in place and also writes the face
// velocity sums u^n + u^{n+1} used for the centre velocity of the CH step.
#include "gpe_plane.hpp"

namespace gpe {

template <typename T, int DIM, bool AXI, int STAGE, int TX, int TY>
__global__ __launch_bounds__(TX* TY) void flow_stage_kernel(FlowArgs<T> A) {
  constexpr int NT = TX * TY;
  constexpr int PX = TX + 3;                  // in-plane X range [-2, TX]
  constexpr int PY = (DIM == 3) ? TY + 3 : 1;  // in-plane Y range [-2, TY]
  constexpr int PLANE = PX * PY;
  constexpr int EY = (DIM == 3) ? PX : 0;     // LDS stride of a +Y step
  // LDS ring slots (3 planes each) and single-plane buffers
  constexpr int S_P = 0, S_UX = 3, S_UY = 6, S_UZ = 9, S_PH = 12, S_ET = 15, S_NU = 18;
  constexpr int S_MU = 21, S_DV = 22, NSLOT = 23;
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

  const T* __restrict__ sp = A.src[0];
  const T* __restrict__ su = A.src[1];
  const T* __restrict__ sv = A.src[2];
  const T* __restrict__ sw = A.src[3];
  const T* __restrict__ phi = A.phi;

  auto slot = [](int k) { return (k + 3) % 3; };

  // Stage plane k (ghost rules applied) into ring slot s.
  auto load_plane = [&](int k, int s) {
    const ZMap<T> z(g, k);
#pragma unroll
    for (int p = 0; p < pm.NPASS; ++p) {
      const int lp = (int)threadIdx.x + p * NT;
      if (lp >= PLANE) continue;
      T vp = T(0), vx = T(0), vy = T(0), vz = T(0), ph = T(0);
      if (pm.ok[p]) {
        vp = sp[z.zc + pm.off_c[p]];
        vx = su[z.zc + pm.off_x[p]] * (pm.sg_x[p] * z.tan);
        if (DIM == 3) vy = sv[z.zc + pm.off_y[p]] * (pm.sg_y[p] * z.tan);
        vz = sw[z.zf + pm.off_c[p]] * (pm.sg_z[p] * z.nrm);
        ph = phi[z.zc + pm.off_c[p]];
      }
      const T eta = eta_of(c, ph);
      const T rho = rho_of(c, ph);
      lds[(S_P + s) * PLANE + lp] = vp;
      lds[(S_UX + s) * PLANE + lp] = vx;
      if (DIM == 3) lds[(S_UY + s) * PLANE + lp] = vy;
      lds[(S_UZ + s) * PLANE + lp] = vz;
      lds[(S_PH + s) * PLANE + lp] = ph;
      lds[(S_ET + s) * PLANE + lp] = eta;
      lds[(S_NU + s) * PLANE + lp] = eta * recip(rho);
    }
  };

  // Chemical potential at LDS position q of plane k (phi ring planes k-1..k+1):
  // mu = 4 a phi (phi^2 - 1) - 6 kappa sum_i w_i (phi_i - phi_c)  (Sec. 2, Sec. 3)
  auto mu_at = [&](int k, int q) -> T {
    const T* F0 = &lds[(S_PH + slot(k)) * PLANE + q];
    const T* Fm = &lds[(S_PH + slot(k - 1)) * PLANE + q];
    const T* Fp = &lds[(S_PH + slot(k + 1)) * PLANE + q];
    const T f = F0[0];
    T rp = T(1), rm = T(1);
    if (AXI) {  // Z is radial: weight every link by its mid-point radius / r_k
      const T rk = T(k) + T(0.5);
      rp = (rk + T(0.5)) / rk;
      rm = (rk - T(0.5)) / rk;
    }
    T lap;
    if (DIM == 2) {
      const T s1 = (F0[1] - f) + (F0[-1] - f) + rp * (Fp[0] - f) + rm * (Fm[0] - f);
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

  // Velocity divergence at LDS position q of plane k (Sec. 3, div stencil);
  // axisymmetric: (1/r) d(r u_r)/dr with face radii k and k+1.
  auto div_at = [&](int k, int q) -> T {
    const T* UX = &lds[(S_UX + slot(k)) * PLANE + q];
    const T* UZ0 = &lds[(S_UZ + slot(k)) * PLANE + q];
    const T* UZp = &lds[(S_UZ + slot(k + 1)) * PLANE + q];
    T d = UX[1] - UX[0];
    if (DIM == 3) {
      const T* UY = &lds[(S_UY + slot(k)) * PLANE + q];
      d += UY[EY] - UY[0];
    }
    if (AXI) {
      const T rk = T(k) + T(0.5);
      d += ((T(k) + T(1)) * UZp[0] - T(k) * UZ0[0]) / rk;
    } else {
      d += UZp[0] - UZ0[0];
    }
    return d;
  };

  // -------- warm-up: planes z0-2 .. z0 -------------------------------------
  load_plane(z0 - 2, slot(z0 - 2));
  load_plane(z0 - 1, slot(z0 - 1));
  load_plane(z0, slot(z0));
  __syncthreads();
  T mu_prev = mu_at(z0 - 1, own);
  T dv_prev = div_at(z0 - 1, own);
  __syncthreads();

  for (int k = z0; k < z1; ++k) {
    load_plane(k + 1, slot(k + 1));
    __syncthreads();

    // mu and div u of plane k on [-1, T-1] (LDS positions 1 .. T+1)
    {
      constexpr int EX_N = TX + 1;
      constexpr int EN = (DIM == 3) ? (TX + 1) * (TY + 1) : TX + 1;
      for (int e = (int)threadIdx.x; e < EN; e += NT) {
        const int ex = e % EX_N, ey = e / EX_N;
        const int q = ((DIM == 3) ? (ey + 1) * PX : 0) + ex + 1;
        lds[S_MU * PLANE + q] = mu_at(k, q);
        lds[S_DV * PLANE + q] = div_at(k, q);
      }
    }
    __syncthreads();

    if (active) {
      const int sm = slot(k - 1), s0 = slot(k), s1 = slot(k + 1);
      const T* P0 = &lds[(S_P + s0) * PLANE + own];
      const T* Pm = &lds[(S_P + sm) * PLANE + own];
      const T* Pp = &lds[(S_P + s1) * PLANE + own];
      const T* UX0 = &lds[(S_UX + s0) * PLANE + own];
      const T* UXm = &lds[(S_UX + sm) * PLANE + own];
      const T* UXp = &lds[(S_UX + s1) * PLANE + own];
      const T* UY0 = &lds[(S_UY + s0) * PLANE + own];
      const T* UYm = &lds[(S_UY + sm) * PLANE + own];
      const T* UYp = &lds[(S_UY + s1) * PLANE + own];
      const T* UZ0 = &lds[(S_UZ + s0) * PLANE + own];
      const T* UZm = &lds[(S_UZ + sm) * PLANE + own];
      const T* UZp = &lds[(S_UZ + s1) * PLANE + own];
      const T* PH0 = &lds[(S_PH + s0) * PLANE + own];
      const T* PHm = &lds[(S_PH + sm) * PLANE + own];
      const T* ET0 = &lds[(S_ET + s0) * PLANE + own];
      const T* ETm = &lds[(S_ET + sm) * PLANE + own];
      const T* ETp = &lds[(S_ET + s1) * PLANE + own];
      const T* NU0 = &lds[(S_NU + s0) * PLANE + own];
      const T* NUm = &lds[(S_NU + sm) * PLANE + own];
      const T* NUp = &lds[(S_NU + s1) * PLANE + own];
      const T* MU = &lds[S_MU * PLANE + own];
      const T* DV = &lds[S_DV * PLANE + own];

      // axisymmetric radii of row k (Z radial): centre r_k, faces R_k = k, R_{k+1}
      const T rk = T(k) + T(0.5);
      const T Rk = T(k), Rk1 = T(k) + T(1);
      const T inv_rk = T(1) / rk;

      // ---- pressure equation at the cell centre ----
      const T pc = P0[0], nuc = NU0[0];
      T diff = T(0.5) * (nuc + NU0[1]) * (P0[1] - pc) - T(0.5) * (nuc + NU0[-1]) * (pc - P0[-1]);
      if (DIM == 3)
        diff += T(0.5) * (nuc + NU0[EY]) * (P0[EY] - pc) - T(0.5) * (nuc + NU0[-EY]) * (pc - P0[-EY]);
      {
        const T fp = T(0.5) * (nuc + NUp[0]) * (Pp[0] - pc);
        const T fm = T(0.5) * (nuc + NUm[0]) * (pc - Pm[0]);
        diff += AXI ? (Rk1 * fp - Rk * fm) * inv_rk : fp - fm;
      }
      const T Lp = -rho_of(c, PH0[0]) * c.cs2 * DV[0] + diff;

      // ---- momentum at an in-plane face (normal A; offset ea, other in-plane
      //      axis B with offset eb in 3-D, Z transverse) ----
      auto face_inplane = [&](const T* UA0, const T* UAm, const T* UAp, const T* UB0, int ea,
                              int eb, T gA) -> T {
        const T ua = UA0[0];
        const T phc = PH0[0], phl = PH0[-ea];
        const T rho_f = T(0.5) * (rho_of(c, phl) + rho_of(c, phc));
        const T eh = ET0[0], el = ET0[-ea];
        // convection
        T C = ua * (UA0[ea] - UA0[-ea]) * T(0.5);
        {
          const T uzb = T(0.25) * ((UZ0[0] + UZ0[-ea]) + (UZp[0] + UZp[-ea]));
          C += uzb * (UAp[0] - UAm[0]) * T(0.5);
        }
        if (DIM == 3) {
          const T ubb = T(0.25) * ((UB0[0] + UB0[-ea]) + (UB0[eb] + UB0[eb - ea]));
          C += ubb * (UA0[eb] - UA0[-eb]) * T(0.5);
        }
        // viscous stress divergence, bulk viscosity eta_b = eta
        T V = T(2) * (eh * (UA0[ea] - ua) - el * (ua - UA0[-ea]));
        {
          const T ep = T(0.25) * ((eh + ETp[0]) + (el + ETp[-ea]));
          const T em = T(0.25) * ((eh + ETm[0]) + (el + ETm[-ea]));
          const T fp = ep * ((UAp[0] - ua) + (UZp[0] - UZp[-ea]));
          const T fm = em * ((ua - UAm[0]) + (UZ0[0] - UZ0[-ea]));
          V += AXI ? (Rk1 * fp - Rk * fm) * inv_rk : fp - fm;
        }
        if (DIM == 3) {
          const T ep = T(0.25) * ((eh + ET0[eb]) + (el + ET0[eb - ea]));
          const T em = T(0.25) * ((eh + ET0[-eb]) + (el + ET0[-eb - ea]));
          const T fp = ep * ((UA0[eb] - ua) + (UB0[eb] - UB0[eb - ea]));
          const T fm = em * ((ua - UA0[-eb]) + (UB0[0] - UB0[-ea]));
          V += fp - fm;
        }
        V += eh * DV[0] - el * DV[-ea];
        // transversely averaged pressure gradient, difference-first
        T G;
        if (DIM == 2) {
          const T d0 = P0[0] - P0[-ea], dp = Pp[0] - Pp[-ea], dm = Pm[0] - Pm[-ea];
          G = (T(4) * d0 + (dp + dm)) * T(1.0 / 6.0);
        } else {
          const T r0 = T(4) * (P0[0] - P0[-ea]) + ((P0[eb] - P0[eb - ea]) + (P0[-eb] - P0[-eb - ea]));
          const T rp = T(4) * (Pp[0] - Pp[-ea]) + ((Pp[eb] - Pp[eb - ea]) + (Pp[-eb] - Pp[-eb - ea]));
          const T rm = T(4) * (Pm[0] - Pm[-ea]) + ((Pm[eb] - Pm[eb - ea]) + (Pm[-eb] - Pm[-eb - ea]));
          G = (T(4) * r0 + (rp + rm)) * T(1.0 / 36.0);
        }
        const T S = -c.sigma * (phc + phl) * (MU[0] - MU[-ea]) * T(0.5);
        const T B = (rho_f - c.rho_ref) * gA;
        return -C + (-G + V + S + B) * recip(rho_f);
      };

      const T LuX = face_inplane(UX0, UXm, UXp, UY0, 1, EY, c.g[0]);
      T LuY = T(0);
      if (DIM == 3) LuY = face_inplane(UY0, UYm, UYp, UX0, EY, 1, c.g[1]);

      // ---- momentum at the Z face between planes k-1 and k ----
      T LuZ = T(0);
      const bool bZ = (k == 0 && g.bc[4] != BC_PERIODIC);
      if (!bZ) {
        const T uz = UZ0[0];
        const T phc = PH0[0], phl = PHm[0];
        const T rho_f = T(0.5) * (rho_of(c, phl) + rho_of(c, phc));
        const T eh = ET0[0], el = ETm[0];
        T C = uz * (UZp[0] - UZm[0]) * T(0.5);
        {
          const T uxb = T(0.25) * ((UX0[0] + UXm[0]) + (UX0[1] + UXm[1]));
          C += uxb * (UZ0[1] - UZ0[-1]) * T(0.5);
        }
        if (DIM == 3) {
          const T uyb = T(0.25) * ((UY0[0] + UYm[0]) + (UY0[EY] + UYm[EY]));
          C += uyb * (UZ0[EY] - UZ0[-EY]) * T(0.5);
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
        {
          const T ep = T(0.25) * ((eh + ET0[1]) + (el + ETm[1]));
          const T em = T(0.25) * ((eh + ET0[-1]) + (el + ETm[-1]));
          const T fp = ep * ((UZ0[1] - uz) + (UX0[1] - UXm[1]));
          const T fm = em * ((uz - UZ0[-1]) + (UX0[0] - UXm[0]));
          V += fp - fm;
        }
        if (DIM == 3) {
          const T ep = T(0.25) * ((eh + ET0[EY]) + (el + ETm[EY]));
          const T em = T(0.25) * ((eh + ET0[-EY]) + (el + ETm[-EY]));
          const T fp = ep * ((UZ0[EY] - uz) + (UY0[EY] - UYm[EY]));
          const T fm = em * ((uz - UZ0[-EY]) + (UY0[0] - UYm[0]));
          V += fp - fm;
        }
        V += eh * DV[0] - el * dv_prev;
        T G;
        if (DIM == 2) {
          G = (T(4) * (P0[0] - Pm[0]) + ((P0[1] - Pm[1]) + (P0[-1] - Pm[-1]))) * T(1.0 / 6.0);
        } else {
          auto row = [&](int o) {
            return T(4) * (P0[o] - Pm[o]) + ((P0[o + 1] - Pm[o + 1]) + (P0[o - 1] - Pm[o - 1]));
          };
          G = (T(4) * row(0) + (row(EY) + row(-EY))) * T(1.0 / 36.0);
        }
        const T S = -c.sigma * (phc + phl) * (MU[0] - mu_prev) * T(0.5);
        const T B = (rho_f - c.rho_ref) * c.g[2];
        LuZ = -C + (-G + V + S + B) * recip(rho_f);
      }

      // ---- Shu-Osher combination of the stage ----
      const bool bX = (i == 0 && g.bc[0] != BC_PERIODIC);
      const bool bY = (DIM == 3) && (j == 0 && g.bc[2] != BC_PERIODIC);
      const size_t ci = ((size_t)k * ny + j) * nx + i;
      const T dt = c.dt;
      T q[4] = {P0[0], UX0[0], (DIM == 3) ? UY0[0] : T(0), UZ0[0]};
      T L[4] = {Lp, LuX, LuY, LuZ};
      T out[4];
      T old[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        if (DIM == 2 && f == 2) continue;
        if (STAGE == 1) {
          out[f] = q[f] + dt * L[f];
        } else {
          old[f] = A.qn[f][ci];
          // Shu-Osher combination in increment form: exact for L = 0
          if (STAGE == 2)
            out[f] = old[f] + T(0.25) * ((q[f] - old[f]) + dt * L[f]);
          else
            out[f] = old[f] + T(2.0 / 3.0) * ((q[f] - old[f]) + dt * L[f]);
        }
      }
      if (bX) out[1] = T(0);
      if (bY) out[2] = T(0);
      if (bZ) out[3] = T(0);
      A.dst[0][ci] = out[0];
      A.dst[1][ci] = out[1];
      if (DIM == 3) A.dst[2][ci] = out[2];
      A.dst[3][ci] = out[3];
      if (STAGE == 3) {
        A.usum[0][ci] = old[1] + out[1];
        if (DIM == 3) A.usum[1][ci] = old[2] + out[2];
        A.usum[2][ci] = old[3] + out[3];
      }
    }
    mu_prev = lds[S_MU * PLANE + own];
    dv_prev = lds[S_DV * PLANE + own];
    __syncthreads();
  }
}

template <typename T, int DIM, bool AXI, int STAGE>
static hipError_t launch_flow_t(const FlowArgs<T>& a, hipStream_t s) {
  constexpr int TX = FlowTile<DIM>::TX, TY = FlowTile<DIM>::TY;
  dim3 grid((a.g.n[0] + TX - 1) / TX, (a.g.n[1] + TY - 1) / TY,
            (a.g.n[2] + a.g.zchunk - 1) / a.g.zchunk);
  hipLaunchKernelGGL((flow_stage_kernel<T, DIM, AXI, STAGE, TX, TY>), grid, dim3(TX * TY), 0, s, a);
  return hipGetLastError();
}

template <typename T, int DIM, bool AXI>
static hipError_t launch_flow_g(const FlowArgs<T>& a, int stage, hipStream_t s) {
  switch (stage) {
    case 1: return launch_flow_t<T, DIM, AXI, 1>(a, s);
    case 2: return launch_flow_t<T, DIM, AXI, 2>(a, s);
    case 3: return launch_flow_t<T, DIM, AXI, 3>(a, s);
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_flow(const FlowArgs<T>& a, int geometry, int stage, hipStream_t s) {
  switch (geometry) {
    case 0: return launch_flow_g<T, 2, false>(a, stage, s);
    case 1: return launch_flow_g<T, 2, true>(a, stage, s);
    case 2: return launch_flow_g<T, 3, false>(a, stage, s);
  }
  return hipErrorInvalidValue;
}

template hipError_t launch_flow<float>(const FlowArgs<float>&, int, int, hipStream_t);
template hipError_t launch_flow<double>(const FlowArgs<double>&, int, int, hipStream_t);

}  // namespace gpe
