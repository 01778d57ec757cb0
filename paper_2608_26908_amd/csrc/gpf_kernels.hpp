// gpf_kernels.hpp -- HIP kernels of the coupled GP phase-field / LBM step.
//
// One step = two z-marching launches over TX x TY tiles of (x, y):
//   k_phi_z    phi^n, mu^n            -> phi^{n+1}          (Eq. PhfGrand, Sec. 2.1)
//   k_mulbm_z  phi^n, phi^{n+1}, mu^n, U^{n-1}, f*^{n-1}
//                                     -> mu^{n+1}, U^n, f*^n (Eq. conc; Eqs. LBMEq_1,
//                                        f^eq, discreteForce, buoyancy, rhovel)
// f buffers hold post-collision, pre-streaming populations as deviations
// f - w_k rho0; streaming is a pull at the start of k_mulbm, with half-way
// bounce-back where the source lies behind a wall.  All buffers are A-B:
// every kernel reads one copy and writes the other.
#pragma once
#include "gpf_device.hpp"

namespace gpf {


// Population k of f^n at cell (x, y, z) = P, as a deviation from w_k rho0:
// pulled from the stored post-collision f* of the upstream cell P - c_k, or,
// when that cell lies behind a wall, the reflected f*_{opp k}(P) (half-way
// bounce-back; the wall sits on the zero-flux face of phi and mu).  The
// test-only moving upper wall of axis 1 adds 6 w_k rho0 c_k . U_wall.
template <int D, int Q, class R>
__device__ __forceinline__ R pull_f(const KP<R>& p, const R* __restrict__ fin, int x, int y, int z,
                                    int64_t P, int k) {
  using L = Lat<Q>;
  int src[3] = {x - L::c(k, 0), y - L::c(k, 1), z - L::c(k, 2)};
  bool in = true;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    if (L::c(k, a) == 0) continue;
    if (src[a] < 0 || src[a] >= p.n[a]) {
      if (p.per[a])
        src[a] = (src[a] + p.n[a]) % p.n[a];
      else
        in = false;
    }
  }
  // each post-collision value is pulled once per step: a streaming
  // (nontemporal) load, as the stores of the new state are streaming stores
  if (in)
    return __builtin_nontemporal_load(&fin[k * p.cells + (int64_t)src[2] * p.sz + (int64_t)src[1] * p.sy + src[0]]);
  R val = fin[Lat<Q>::opp(k) * p.cells + P];
  if (L::c(k, 1) < 0 && !p.per[1] && y - L::c(k, 1) >= p.n[1])
    val += R(6 * L::w(k)) * p.rho0 * R(L::c(k, 0)) * p.lid_u;
  return val;
}

// Element u + l of a buffer, u wave-uniform and l a lane's own non-negative
// offset: the uniform part is formed in scalar registers and the access is a
// global load or store with a scalar base and a 32-bit lane offset.
template <class T>
__device__ __forceinline__ T* lane_at(T* base, int64_t u, int l) {
  using C = typename std::conditional<std::is_const<T>::value, const char, char>::type;
  return reinterpret_cast<T*>(reinterpret_cast<C*>(base + u) + (uint32_t)l * (uint32_t)sizeof(T));
}

// Source columns of the pulls of one lane along x, fixed for a z-marching
// thread: xs[1 - c_x] is the column of the cell P - c_k (wrapped on a
// periodic axis, clamped at a wall) and xw[1 - c_x] says it lies behind a wall.
struct PullX {
  int xs[3];
  bool xw[3];
};
__device__ __forceinline__ PullX pull_x(int x, int n0, int per0) {
  PullX q;
  q.xs[1] = x;
  q.xw[1] = false;
  q.xw[0] = !per0 && x - 1 < 0;
  q.xw[2] = !per0 && x + 1 >= n0;
  q.xs[0] = (x - 1 < 0) ? (per0 ? x - 1 + n0 : 0) : x - 1;
  q.xs[2] = (x + 1 >= n0) ? (per0 ? x + 1 - n0 : n0 - 1) : x + 1;
  return q;
}

// The populations f^n of the cell (x, y, z) for a wave whose lanes share the
// row y and plane z (what pull_f does cell by cell): the source row and plane
// of population k, and with them a wall between source and cell along y or z,
// are the same on every lane, so they are decided with scalar arithmetic and
// only the x walls of the grid's first and last column differ between lanes.
template <int D, int Q, class R>
__device__ __forceinline__ void pull_row(const KP<R>& p, const R* __restrict__ fin, int x, int y, int z,
                                         const PullX& px, R (&f)[Q]) {
  using L = Lat<Q>;
  const int64_t own = (int64_t)z * p.sz + (int64_t)y * p.sy;
  // source row and plane of population k; false when behind a y or z wall
  auto src = [&](int k, int64_t& row) -> bool {
    int ys = y - L::c(k, 1), zs = (D == 3) ? z - L::c(k, 2) : z;
    bool in = true;
    if (ys < 0 || ys >= p.n[1]) {
      if (p.per[1])
        ys += (ys < 0) ? p.n[1] : -p.n[1];
      else
        in = false;
    }
    if (D == 3 && (zs < 0 || zs >= p.n[2])) {
      if (p.per[2])
        zs += (zs < 0) ? p.n[2] : -p.n[2];
      else
        in = false;
    }
    row = (int64_t)zs * p.sz + (int64_t)ys * p.sy;
    return in;
  };
  // reflected population at the cell itself (half-way bounce-back), plus the
  // moving-lid term where the source lies above the upper y wall
  auto bounce = [&](int k) -> R {
    R val = *lane_at(fin, (int64_t)L::opp(k) * p.cells + own, x);
    if (L::c(k, 1) < 0 && !p.per[1] && y - L::c(k, 1) >= p.n[1])
      val += R(6 * L::w(k)) * p.rho0 * R(L::c(k, 0)) * p.lid_u;
    return val;
  };
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    int64_t row;
    if (src(k, row))
      f[k] = __builtin_nontemporal_load(lane_at(fin, (int64_t)k * p.cells + row, px.xs[1 - L::c(k, 0)]));
    else
      f[k] = bounce(k);
  }
  // lanes whose x source lies behind a wall (the tiles at x = 0 and n0 - 1)
#pragma unroll
  for (int side = 0; side < 3; side += 2) {
    if (px.xw[side]) {
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        int64_t row;
        if (1 - L::c(k, 0) == side && src(k, row)) f[k] = bounce(k);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Phase field: active set, right-hand side, projection.
// ---------------------------------------------------------------------------
// Active set of a cell: bit b set when phase b is non-zero somewhere in the
// 9/19-point neighbourhood v[phase][dz+1][dy+1][dx+1].
// Phase b is non-zero somewhere exactly when its largest value over the
// neighbourhood is positive (one max per value instead of a compare and a
// select).
template <int D, int N, class R>
__device__ __forceinline__ unsigned active_of(const R (&v)[N][3][3][3]) {
  unsigned active = 0u;
#pragma unroll
  for (int b = 0; b < N; ++b) {
    R m = v[b][1][1][1];
#pragma unroll
    for (int dz = (D == 3 ? -1 : 0); dz <= (D == 3 ? 1 : 0); ++dz)
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          if (dx != 0 && dy != 0 && dz != 0) continue;
          if (dx == 0 && dy == 0 && dz == 0) continue;
          m = fmax(m, v[b][dz + 1][dy + 1][dx + 1]);
        }
    if (m > R(0)) active |= 1u << b;
  }
  return active;
}

// Right-hand side R_a of Eq. (PhfGrand) (tau eps dphi_a/dt = R_a before the
// constraint) for every phase, from phi^n on the neighbourhood v (walls
// mirrored, periodic axes wrapped; the cube corners are not used) and mu^n:
//   R_a = eps [div J_a - sum_b dA_ab/dq(q_ab) . grad phi_b] - dW/dphi_a / eps
//         - sum_b psi^b dh_b/dphi_a,
// J_a = -sum_b phi_b,f dA_ab/dq(q_ab,f) on faces (none on wall faces).
template <int D, int N, int NC, class R>
__device__ __forceinline__ void pf_rhs(const KP<R>& p, const R (&v)[N][3][3][3],
                                       const R* __restrict__ mu, int x, int y, int z, R tshift,
                                       R (&Rv)[N]) {
  const int64_t P = (int64_t)z * p.sz + (int64_t)y * p.sy + x;
  const int pos[3] = {x, y, z};
  const R idx = R(1) / p.dx;
  const R ih2 = R(0.5) / p.dx;
  // central difference along e at X = P + o (o within the neighbourhood)
  auto gc = [&](int b, int ox, int oy, int oz, int e) -> R {
    int op[3] = {ox, oy, oz}, om[3] = {ox, oy, oz};
    op[e] += 1;
    om[e] -= 1;
    return (v[b][op[2] + 1][op[1] + 1][op[0] + 1] - v[b][om[2] + 1][om[1] + 1][om[0] + 1]) * ih2;
  };

  R div[N];
#pragma unroll
  for (int b = 0; b < N; ++b) div[b] = R(0);

  // face fluxes J_a = -sum_b phi_b,f dA_ab/dq(q_ab,f), q = phi_a grad phi_b - phi_b grad phi_a
#pragma unroll
  for (int a = 0; a < D; ++a) {
#pragma unroll
    for (int s = -1; s <= 1; s += 2) {
      const bool wall = !p.per[a] && ((s < 0 && pos[a] == 0) || (s > 0 && pos[a] == p.n[a] - 1));
      if (wall) continue;
      int o[3] = {0, 0, 0};
      o[a] = s;
      R pf[N], gf[N][D];
#pragma unroll
      for (int b = 0; b < N; ++b) {
        const R vP = v[b][1][1][1];
        const R vQ = v[b][o[2] + 1][o[1] + 1][o[0] + 1];
        pf[b] = R(0.5) * (vP + vQ);
#pragma unroll
        for (int e = 0; e < D; ++e) {
          if (e == a)
            gf[b][e] = R(s) * (vQ - vP) * idx;
          else
            gf[b][e] = R(0.5) * (gc(b, 0, 0, 0, e) + gc(b, o[0], o[1], o[2], e));
        }
      }
      R J[N];
#pragma unroll
      for (int b = 0; b < N; ++b) J[b] = R(0);
#pragma unroll
      for (int al = 0; al < N; ++al)
#pragma unroll
        for (int be = al + 1; be < N; ++be) {
          R q[D], g[D];
#pragma unroll
          for (int e = 0; e < D; ++e) q[e] = pf[al] * gf[be][e] - pf[be] * gf[al][e];
          dAdq<D, R, R>(q, p.gamma[al][be], p.delta[al][be], p.qmin2, g);
          J[al] -= pf[be] * g[a];
          J[be] += pf[al] * g[a];
        }
#pragma unroll
      for (int b = 0; b < N; ++b) div[b] += R(s) * J[b] * idx;
    }
  }

  // cell-centre terms
  R ph[N], g0[N][D];
#pragma unroll
  for (int b = 0; b < N; ++b) {
    ph[b] = v[b][1][1][1];
#pragma unroll
    for (int e = 0; e < D; ++e) g0[b][e] = gc(b, 0, 0, 0, e);
  }
  R cell[N];
#pragma unroll
  for (int b = 0; b < N; ++b) cell[b] = R(0);
#pragma unroll
  for (int al = 0; al < N; ++al)
#pragma unroll
    for (int be = al + 1; be < N; ++be) {
      R q[D], g[D];
#pragma unroll
      for (int e = 0; e < D; ++e) q[e] = ph[al] * g0[be][e] - ph[be] * g0[al][e];
      dAdq<D, R, R>(q, p.gamma[al][be], p.delta[al][be], p.qmin2, g);
#pragma unroll
      for (int e = 0; e < D; ++e) {
        cell[al] += g[e] * g0[be][e];
        cell[be] -= g[e] * g0[al][e];
      }
    }

  // grand potentials psi^b(mu, T) = -1/2 mu.chi.mu - mu.(c0[b] + mT[b] (T - T_E)) + dS[b] (T - T_E)
  R m[NC];
#pragma unroll
  for (int i = 0; i < NC; ++i) m[i] = p.mu_ref[i] + mu[i * p.cells + P];
  const R tdev = (p.G != R(0)) ? p.G * (R(pos[p.pull_axis]) - tshift) : p.tdev_iso;
  R ps[N];
#pragma unroll
  for (int b = 0; b < N; ++b) {
    R r = R(0);
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      R chimu = R(0);
#pragma unroll
      for (int j = 0; j < NC; ++j) chimu += p.chi[i][j] * m[j];
      r += -R(0.5) * m[i] * chimu - m[i] * (p.c0[b][i] + p.mT[b][i] * tdev);
    }
    ps[b] = r + p.dS[b] * tdev;
  }

#pragma unroll
  for (int al = 0; al < N; ++al) {
    R dW = R(0);
#pragma unroll
    for (int be = 0; be < N; ++be) {
      if (be == al) continue;
      if (p.potential == 0)
        dW += R(1.6211389382774044) * p.gamma[al][be] * ph[be];  // 16 / pi^2
      else
        dW += R(18) * p.gamma[al][be] * ph[al] * ph[be] * ph[be];
    }
    R drive = R(0);
#pragma unroll
    for (int be = 0; be < N; ++be) drive += ps[be] * dh<N, R>(ph, be, al);
    Rv[al] = p.eps * (div[al] - cell[al]) - dW * p.ieps - drive;
  }
}

// phi^{n+1} of a cell from its neighbourhood v and mu^n: unchanged when one
// phase is active (bulk, returned true), else the projection of
// phi + dt/(tau eps) R over the active phases onto the simplex.  act_out, if
// not null, receives the cell's active set.
template <int D, int N, int NC, class R>
__device__ __forceinline__ bool phi_from_stencil(const KP<R>& p, const R (&v)[N][3][3][3],
                                                 const R* __restrict__ mu, int x, int y, int z,
                                                 R tshift, R (&res)[N], uint8_t* __restrict__ act_out) {
  const unsigned active = active_of<D, N, R>(v);
  if (act_out) *act_out = (uint8_t)active;
  if (__builtin_popcount(active) <= 1) {  // bulk: phi unchanged
#pragma unroll
    for (int b = 0; b < N; ++b) res[b] = v[b][1][1][1];
    return true;
  }
  R Rv[N], vv[N];
  pf_rhs<D, N, NC, R>(p, v, mu, x, y, z, tshift, Rv);
#pragma unroll
  for (int b = 0; b < N; ++b) vv[b] = v[b][1][1][1] + p.rate * Rv[b];
  R theta;
  project_masked<N, R>(active, vv, res, theta);
  return false;
}

// ---------------------------------------------------------------------------
// mu^{n+1}, U^n and the post-collision populations of cell (x, y, z), given
// the values it reads around itself:
//   ph1n[0] / mun[0]: phi^{n+1} / mu^n at the cell, ph1n[1 + 2a + s] / mun[..]
//   at its -e_a (s = 0) and +e_a (s = 1) neighbours (wrapped on periodic
//   axes; never used across walls); uc: U^{n-1} at the cell; un[a][s]: the
//   a-component of U^{n-1} at those neighbours; ph0: phi^n at the cell.
// The populations are pulled from fin (the previous post-collision f*).
// ---------------------------------------------------------------------------
// SH: the shrinkage force is on (a separate instance keeps the registers of
// the common case unchanged)
// T - T_E of a cell at pull-axis coordinate c, step shift ts
template <class R>
__device__ __forceinline__ R tdev_at(const KP<R>& p, int c, R ts) {
  return (p.G != R(0)) ? p.G * (R(c) - ts) : p.tdev_iso;
}

// MT: the equilibrium compositions depend on T (some mT != 0); a separate
// instance keeps the registers of the common case
template <int D, int Q, int N, int NC, class R, bool SH, bool MT>
__device__ __forceinline__ void mulbm_core(const KP<R>& p, int x, int y, int z, const PullX& px, R ts0,
                                           const R (&ph1n)[2 * D + 1][N],
                                           const R (&mun)[2 * D + 1][NC], const R (&uc)[D],
                                           const R (&un)[D][2], const R (&ph0)[N],
                                           const R* __restrict__ fin, R* __restrict__ mu_out,
                                           R* __restrict__ u_out, R* __restrict__ fout,
                                           R* __restrict__ dr_out) {
  using L = Lat<Q>;
  const int64_t own = (int64_t)z * p.sz + (int64_t)y * p.sy;  // the cell is own + x
  const int pos[3] = {x, y, z};
  // T^n - T_E at the cell and at its neighbours (slots of ph1n); only the
  // neighbours along the pull axis differ from the cell
  const int pa = p.pull_axis;
  const R tdc = MT ? tdev_at(p, pos[pa], ts0) : R(0);
  auto tdev_slot = [&](int slot) -> R {
    if constexpr (!MT) return R(0);
    if (slot == 0) return tdc;
    const int a = (slot - 1) / 2;
    if (a != pa) return tdc;
    return tdev_at(p, nb_field(pos[a], ((slot - 1) & 1) ? 1 : -1, p.n[a], p.per[a]), ts0);
  };

  // pull streaming of the previous post-collision populations: issued first,
  // so the loads are in flight during the chemical-potential update, where
  // that costs no occupancy (FP32, two phases, one solute; elsewhere the
  // populations held through the update take the kernel past a register
  // threshold)
  constexpr bool EARLY = !SH && !MT && N == 2 && NC == 1 && sizeof(R) == 4;
  R f[L::Q];
  if constexpr (EARLY) pull_row<D, Q, R>(p, fin, x, y, z, px, f);

  // per-cell quantities at phi^{n+1}: c* = sum h C(mu^n, T^n), M = sum phi D chi
  auto quant = [&](int slot, R (&M)[NC][NC], R (&cs)[NC]) {
    const R td = tdev_slot(slot);
    R ph[N], h[N];
#pragma unroll
    for (int b = 0; b < N; ++b) ph[b] = ph1n[slot][b];
    interp_h<N, R>(ph, h);
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      cs[i] = R(0);
#pragma unroll
      for (int k = 0; k < NC; ++k) M[i][k] = R(0);
    }
#pragma unroll
    for (int b = 0; b < N; ++b) {
#pragma unroll
      for (int i = 0; i < NC; ++i) {
        R C = p.c0s[b][i];
        if constexpr (MT) C += p.mT[b][i] * td;
#pragma unroll
        for (int k = 0; k < NC; ++k) C += p.chi[i][k] * mun[slot][k];
        cs[i] += h[b] * C;
#pragma unroll
        for (int k = 0; k < NC; ++k) M[i][k] += ph[b] * p.D[b][i] * p.chi[i][k];
      }
    }
  };

  R MP[NC][NC], cP[NC];
  quant(0, MP, cP);
  R divJ[NC];
#pragma unroll
  for (int i = 0; i < NC; ++i) divJ[i] = R(0);
  const R conv = p.conv;  // lattice velocity -> phase-field units
  const R idx = p.idx;
#pragma unroll
  for (int a = 0; a < D; ++a) {
#pragma unroll
    for (int si = 0; si < 2; ++si) {
      const int s = si ? 1 : -1;
      const bool wall = !p.per[a] && ((s < 0 && pos[a] == 0) || (s > 0 && pos[a] == p.n[a] - 1));
      if (wall) continue;
      const int slot = 1 + 2 * a + si;
      R MQ[NC][NC], cQ[NC];
      quant(slot, MQ, cQ);
      const R uf = R(0.5) * (uc[a] + un[a][si]) * conv;
#pragma unroll
      for (int i = 0; i < NC; ++i) {
        R JD = R(0);
#pragma unroll
        for (int k = 0; k < NC; ++k)
          JD += -R(0.5) * (MP[i][k] + MQ[i][k]) * (R(s) * (mun[slot][k] - mun[0][k]) * idx);
        const R JA = uf * R(0.5) * (cP[i] + cQ[i]);
        divJ[i] += R(s) * (JD + JA) * idx;
      }
    }
  }
  R ph1[N], h0[N], h1[N];
#pragma unroll
  for (int b = 0; b < N; ++b) ph1[b] = ph1n[0][b];
  interp_h<N, R>(ph0, h0);
  interp_h<N, R>(ph1, h1);
  R Dl[NC];
#pragma unroll
  for (int i = 0; i < NC; ++i) Dl[i] = -p.dt * divJ[i];
  // dh/dt source with C at T^n, and the dT/dt term of Eq. (conc) over the
  // step, -sum_b h_b^{n+1} (C^b(mu^n, T^{n+1}) - C^b(mu^n, T^n)) = -sum_b
  // h_b^{n+1} mT[b] (T^{n+1} - T^n)
  const R td0 = tdev_slot(0);
  R sh = R(0);
#pragma unroll
  for (int b = 0; b < N; ++b) {
    sh += h1[b];
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      R C = p.c0s[b][i];
      if constexpr (MT) C += p.mT[b][i] * td0;
#pragma unroll
      for (int k = 0; k < NC; ++k) C += p.chi[i][k] * mun[0][k];
      Dl[i] -= C * (h1[b] - h0[b]);
      if constexpr (MT) Dl[i] -= h1[b] * (p.mT[b][i] * p.dtdev);
    }
  }
  R mn[NC];
  if (NC == 1) {
    mn[0] = mun[0][0] + Dl[0] / (sh * p.chi[0][0]);
  } else {
    const R a11 = sh * p.chi[0][0], a12 = sh * p.chi[0][1];
    const R a21 = sh * p.chi[1][0], a22 = sh * p.chi[1][NC - 1];
    const R det = a11 * a22 - a12 * a21;
    mn[0] = mun[0][0] + (a22 * Dl[0] - a12 * Dl[NC - 1]) / det;
    mn[NC - 1] = mun[0][NC - 1] + (-a21 * Dl[0] + a11 * Dl[NC - 1]) / det;
  }
#pragma unroll
  for (int i = 0; i < NC; ++i) __builtin_nontemporal_store(mn[i], lane_at(mu_out, i * p.cells + own, x));

  // ---- LBM: pull streaming of the previous post-collision populations ----
  if constexpr (!EARLY) pull_row<D, Q, R>(p, fin, x, y, z, px, f);
  // moments (deviation storage: rho = rho0 + sum f~, momentum = sum f~ c)
  R dr = R(0), mom[D];
#pragma unroll
  for (int a = 0; a < D; ++a) mom[a] = R(0);
#pragma unroll
  for (int k = 0; k < L::Q; ++k) {
    dr += f[k];
#pragma unroll
    for (int a = 0; a < D; ++a)
      if (L::c(k, a) != 0) mom[a] += R(L::c(k, a)) * f[k];
  }
  const R rho = p.rho0 + dr;
  if (dr_out) *lane_at(dr_out, own, x) = dr;  // kept for the adjoint sweep
  const R phil = ph1[N - 1];
  R bsum = R(0);
#pragma unroll
  for (int i = 0; i < NC; ++i) {
    R Cl = p.c0s[N - 1][i];
    if constexpr (MT) Cl += p.mT[N - 1][i] * (td0 + p.dtdev);  // the liquid at T^{n+1}
#pragma unroll
    for (int k = 0; k < NC; ++k) Cl += p.chi[i][k] * mn[k];
    bsum += p.gbeta[i] * (Cl - p.c_ref[i]);
  }
  R FB[D];
#pragma unroll
  for (int a = 0; a < D; ++a) FB[a] = R(0);
  FB[p.grav_axis] = -rho * phil * bsum * p.grav_sign;
  if constexpr (SH) {
    // shrinkage, Eq. (shrinkage): eta_b (phi^{n+1}_b - phi^n_b) along the unit
    // normal of phi^{n+1}_b (central differences over the 7-point values held
    // for the mu update; walls mirrored), per lattice step
#pragma unroll
    for (int b = 0; b < N; ++b) {
      if (p.eta[b] == R(0)) continue;
      R g[D], gg = R(0);
#pragma unroll
      for (int a = 0; a < D; ++a) {
        g[a] = (ph1n[2 + 2 * a][b] - ph1n[1 + 2 * a][b]) / (R(2) * p.dx);
        gg += g[a] * g[a];
      }
      if (gg > p.qmin2) {
        const R s = p.eta[b] * (ph1n[0][b] - ph0[b]) / gsqrt(gg);
#pragma unroll
        for (int a = 0; a < D; ++a) FB[a] += s * g[a];
      }
    }
  }
  const R sol = (R(1) - phil) * (R(1) - phil);
  R u[D], F[D];
  const R iu = (phil != R(0)) ? R(1) / (rho * (R(1) + R(0.5) * p.kappa * sol)) : R(0);
#pragma unroll
  for (int a = 0; a < D; ++a) {
    u[a] = (mom[a] + R(0.5) * FB[a]) * iu;
    F[a] = FB[a] - p.kappa * rho * sol * u[a];
  }
  R uu = R(0), uF = R(0);
#pragma unroll
  for (int a = 0; a < D; ++a) {
    uu += u[a] * u[a];
    uF += u[a] * F[a];
  }
  const R pref = p.guo;
#pragma unroll
  for (int k = 0; k < L::Q; ++k) {
    R cu = R(0), cF = R(0);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      if (L::c(k, a) != 0) {
        cu += R(L::c(k, a)) * u[a];
        cF += R(L::c(k, a)) * F[a];
      }
    }
    const R wk = R(L::w(k));
    const R feq = wk * (dr + rho * (R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu));
    const R S = pref * wk * (R(3) * (cF - uF) + R(9) * cu * cF);
    __builtin_nontemporal_store(f[k] - (f[k] - feq) * p.omega + S, lane_at(fout, k * p.cells + own, x));
  }
#pragma unroll
  for (int a = 0; a < D; ++a) __builtin_nontemporal_store(u[a], lane_at(u_out, a * p.cells + own, x));
}

// coordinate along one axis of a tile-halo cell: periodic axes wrap, walls
// clamp (values across a wall are never used: wall faces carry no flux)
__device__ __forceinline__ int wrap_or_clamp(int v, int n, int per) {
  if (per) return ((v % n) + n) % n;
  return v < 0 ? 0 : (v >= n ? n - 1 : v);
}

// Tile of a z-marching block.  Work-groups are dealt to the 8 XCDs
// round-robin; renumbering gives each XCD a contiguous range of tiles, so
// tiles that are neighbours in y and z share its L2.
struct Tile {
  int x0, y0, z0, z1;
  unsigned lb;  // logical tile index: x fastest, then y, then the chunk along z
};
__device__ __forceinline__ Tile tile_at(unsigned lb, int tiles_x, int tiles_y, int tx, int ty, int zc,
                                        int nz, int D) {
  Tile t;
  t.lb = lb;
  t.x0 = (int)(lb % (unsigned)tiles_x) * tx;
  t.y0 = (int)((lb / (unsigned)tiles_x) % (unsigned)tiles_y) * ty;
  const int tz = (int)(lb / ((unsigned)tiles_x * (unsigned)tiles_y));
  t.z0 = (D == 3) ? tz * zc : 0;
  t.z1 = (D == 3) ? min(t.z0 + zc, nz) : 1;
  return t;
}
__device__ __forceinline__ Tile tile_of(int tiles_x, int tiles_y, int tx, int ty, int zc, int nz,
                                        int D) {
  const unsigned nb = gridDim.x, b = blockIdx.x;
  const unsigned per8 = nb / 8u;
  const unsigned lb = (b < per8 * 8u) ? (b % 8u) * per8 + b / 8u : b;
  return tile_at(lb, tiles_x, tiles_y, tx, ty, zc, nz, D);
}

// ---------------------------------------------------------------------------
// Phase field, z-marching: a block owns a TX x TY tile and walks along z
// through planes [z0, z1).  phi^n of the tile plus a one-cell halo is kept in
// a four-slot LDS ring (planes z-1, z, z+1 in use, z+2 being filled), so every
// phi^n value is read from memory once per block and the 9/19-point stencil
// reads LDS.  The plane two ahead is fetched into registers before a plane is
// computed and stored to the ring after it, so its loads are in flight during
// the computation; one barrier per plane.
// ---------------------------------------------------------------------------
// One block's walk through the planes of its tile T (the body of k_phi_z and
// k_phi_zl).  was_bulk: phi_out, which still holds phi^{n-1}, already holds
// phi^n on every cell of T.  Ends in a barrier after the last read of the
// ring.
template <int D, int N, int NC, class R, int TX, int TY, bool ACT, class Ring>
__device__ __forceinline__ void phi_walk(const KP<R>& p, const R* __restrict__ phi, const R* __restrict__ mu,
                                         R* __restrict__ phi_out, bool was_bulk, uint8_t* __restrict__ bulk_out,
                                         uint8_t* __restrict__ act_out, R tshift, const Tile& T, Ring& ring) {
  constexpr int HX = TX + 2, HY = TY + 2, HC = HX * HY;
  constexpr int NT = TX * TY, PER = (HC + NT - 1) / NT;  // halo-tile cells per thread
  const int tid = threadIdx.x;
  const int lx = tid % TX, ly = tid / TX;
  const int x = T.x0 + lx, y = T.y0 + ly;
  const bool own = x < p.n[0] && y < p.n[1];
  const int c0 = (ly + 1) * HX + (lx + 1);
  int all_bulk = 1;

  // in-plane offsets of this thread's halo-tile cells (fixed along z)
  int64_t hoff[PER];
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const int i = min(tid + r * NT, HC - 1);
    const int gx = wrap_or_clamp(T.x0 - 1 + i % HX, p.n[0], p.per[0]);
    const int gy = wrap_or_clamp(T.y0 - 1 + i / HX, p.n[1], p.per[1]);
    hoff[r] = (int64_t)gy * p.sy + gx;
  }
  R pre[PER][N];
  auto fetch = [&](int zz) {
    const int64_t zo = (D == 3) ? (int64_t)wrap_or_clamp(zz, p.n[2], p.per[2]) * p.sz : 0;
#pragma unroll
    for (int r = 0; r < PER; ++r)
      if (tid + r * NT < HC)
#pragma unroll
        for (int q = 0; q < N; ++q) pre[r][q] = phi[q * p.cells + zo + hoff[r]];
  };
  auto store = [&](int slot) {
#pragma unroll
    for (int r = 0; r < PER; ++r)
      if (tid + r * NT < HC)
#pragma unroll
        for (int q = 0; q < N; ++q) ring[slot][q][tid + r * NT] = pre[r][q];
  };
  auto update = [&](int z, int sm, int s0, int sp) {
    if (!own) return;
    int xq = x, yq = y;  // opaque per plane, as in k_mulbm_z
    asm volatile("" : "+v"(xq), "+v"(yq));
    R v[N][3][3][3];
    const int sl[3] = {sm, s0, sp};
#pragma unroll
    for (int dz = (D == 3 ? -1 : 0); dz <= (D == 3 ? 1 : 0); ++dz)
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          if (dx != 0 && dy != 0 && dz != 0) continue;
#pragma unroll
          for (int q = 0; q < N; ++q) v[q][dz + 1][dy + 1][dx + 1] = ring[sl[dz + 1]][q][c0 + dy * HX + dx];
        }
    R res[N];
    uint8_t* ap = nullptr;
    if constexpr (ACT) ap = act_out + (int64_t)z * p.sz + (uint32_t)(yq * (int)p.sy + xq);  // a plane < 2^32 cells
    const bool bulk = phi_from_stencil<D, N, NC, R>(p, v, mu, xq, yq, z, tshift, res, ap);
    all_bulk &= bulk ? 1 : 0;
    if (was_bulk && bulk) return;
    const int64_t P = (int64_t)z * p.sz + (int64_t)yq * p.sy + xq;
#pragma unroll
    for (int q = 0; q < N; ++q) __builtin_nontemporal_store(res[q], &phi_out[q * p.cells + P]);
  };
  auto record_bulk = [&]() {
    const int b = __syncthreads_and(all_bulk);
    if (bulk_out && tid == 0) bulk_out[T.lb] = (uint8_t)b;
  };

  if (D == 2) {
    fetch(0);
    store(0);
    __syncthreads();
    update(0, 0, 0, 0);
    record_bulk();
    return;
  }
  // ring slot of plane zz: (zz - z0 + 1) mod 4
  fetch(T.z0 - 1);
  store(0);
  fetch(T.z0);
  store(1);
  fetch(T.z0 + 1);
  store(2);
  fetch(T.z0 + 2);
  __syncthreads();
  for (int z = T.z0; z < T.z1; ++z) {
    const int k = z - T.z0;
    update(z, k & 3, (k + 1) & 3, (k + 2) & 3);
    if (z + 1 < T.z1) {
      // plane z+2 goes to the slot of plane z-2, which every thread finished
      // reading before the previous barrier
      store((k + 3) & 3);
      if (z + 2 < T.z1) fetch(z + 3);
      __syncthreads();
    }
  }
  record_bulk();
}

// Bulk flag of the tile at neighbour offset i (0..26: dx, dy, dz in -1..1,
// x fastest) of logical tile lb in a grid of nt[0] x nt[1] x nt[2] tiles;
// periodic axes wrap, and a tile beyond a wall counts as bulk (no stencil
// reaches across a wall).
__device__ __forceinline__ int bulk_flag_at(const uint8_t* __restrict__ bulk, unsigned lb, int i, const int nt[3],
                                            const int per[3], int D) {
  const int d[3] = {i % 3 - 1, (i / 3) % 3 - 1, i / 9 - 1};
  int t3[3] = {(int)(lb % (unsigned)nt[0]), (int)((lb / (unsigned)nt[0]) % (unsigned)nt[1]),
               (int)(lb / (unsigned)(nt[0] * nt[1]))};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    t3[a] += d[a];
    if (t3[a] < 0 || t3[a] >= nt[a]) {
      if (a < D && per[a])
        t3[a] += (t3[a] < 0) ? nt[a] : -nt[a];
      else
        return 1;
    }
  }
  return bulk[t3[0] + nt[0] * (t3[1] + nt[1] * t3[2])];
}

template <int D, int N, int NC, class R, int TX, int TY, bool ACT>
__global__ void __launch_bounds__(TX * TY)
k_phi_z(KP<R> p, const R* __restrict__ phi, const R* __restrict__ mu, R* __restrict__ phi_out,
        const uint8_t* __restrict__ bulk_in, uint8_t* __restrict__ bulk_out, uint8_t* __restrict__ act_out,
        R tshift, int tiles_x, int tiles_y, int zc) {
  constexpr int HX = TX + 2, HY = TY + 2, HC = HX * HY;
  constexpr int NS = (D == 3) ? 4 : 1;
  __shared__ R ring[NS][N][HC];
  const Tile T = tile_of(tiles_x, tiles_y, TX, TY, zc, p.n[2], D);
  const int tid = threadIdx.x;
  // Bulk history (both null when phi_out is not the buffer that held phi^{n-1}),
  // one flag per block (logical tile index): bulk_in[block] says every cell of
  // this block's tile and planes was bulk in the step that produced phi^n from
  // phi^{n-1}, so phi_out, which still holds phi^{n-1}, already holds phi^n
  // there, and a cell that is bulk again (phi^{n+1} = phi^n) need not be
  // stored.  bulk_out[block] records the same for this step.
  // ACT (recomputation for the adjoint): act_out receives each cell's active
  // set of phases, which the reverse of the step reads instead of phi^n's
  // stencil (an instance of its own keeps the registers of the common case)
  if (bulk_in && (D == 3 || p.cells > ((int64_t)1 << 18))) {
    // If this block and every block its stencils reach (the 26 around it, none
    // beyond a wall) were bulk in that step, phi^n = phi^{n-1} on every stencil
    // the block evaluates, so each cell has its previous active set and is
    // bulk again: phi_out already holds phi^{n+1} = phi^n, nothing to do.  (On
    // small 2D grids, whose one-plane blocks make a launch of a few
    // microseconds, the flag loads cost what they save.)
    int ok = 1;
    if (tid < 27) {
      const int nt[3] = {tiles_x, tiles_y, (int)(gridDim.x / (unsigned)(tiles_x * tiles_y))};
      ok = bulk_flag_at(bulk_in, T.lb, tid, nt, p.per, D);
    }
    if (__syncthreads_and(ok)) {
      if (bulk_out && tid == 0) bulk_out[T.lb] = 1;
      return;
    }
  }
  phi_walk<D, N, NC, R, TX, TY, ACT>(p, phi, mu, phi_out, bulk_in && bulk_in[T.lb], bulk_out, act_out, tshift, T,
                                     ring);
}

// ---------------------------------------------------------------------------
// Phase field over a list of tiles (3D grids with the bulk history on).  On a
// grid that is mostly bulk nearly every block of a k_phi_z launch finds its
// neighbourhood bulk and returns, yet the launch still pays the dispatch of
// all of them.
// k_phi_todo checks every tile's neighbourhood, one thread per tile, sets the
// flag of each tile it skips and appends the others to a list; k_phi_zl,
// launched with a grid of resident blocks, walks the listed tiles.  Each XCD
// walks a contiguous part of the list (whose waves append in about the order
// of the tiles), so tiles that are neighbours share its L2 as in k_phi_z.
// count is the length of the list; it starts at zero, and the step's
// k_mulbm_z, which runs after k_phi_zl, clears it for the next step.
// ---------------------------------------------------------------------------
template <int D>
__global__ void __launch_bounds__(256)
k_phi_todo(const uint8_t* __restrict__ bulk_in, uint8_t* __restrict__ bulk_out, unsigned* __restrict__ list,
           unsigned* __restrict__ count, int tiles_x, int tiles_y, int tiles_z, int per0, int per1, int per2) {
  const unsigned nb = (unsigned)tiles_x * (unsigned)tiles_y * (unsigned)tiles_z;
  const unsigned lb = blockIdx.x * 256u + threadIdx.x;
  bool need = false;
  if (lb < nb) {
    const int nt[3] = {tiles_x, tiles_y, tiles_z}, per[3] = {per0, per1, per2};
    int ok = 1;
#pragma unroll
    for (int i = 0; i < 27; ++i) ok &= bulk_flag_at(bulk_in, lb, i, nt, per, D);
    if (ok)
      bulk_out[lb] = 1;
    else
      need = true;
  }
  // one atomic per wave; the wave's listed tiles take consecutive slots
  const unsigned long long m = __ballot(need);
  const unsigned lane = __lane_id();
  unsigned base = 0;
  if (m && lane == 0) base = atomicAdd(count, (unsigned)__popcll(m));
  base = __shfl(base, 0);
  const unsigned slot = base + (unsigned)__popcll(m & ((1ull << lane) - 1ull));
  if (need && slot < nb) list[slot] = lb;
}

template <int D, int N, int NC, class R, int TX, int TY>
__global__ void __launch_bounds__(TX * TY)
k_phi_zl(KP<R> p, const R* __restrict__ phi, const R* __restrict__ mu, R* __restrict__ phi_out,
         const uint8_t* __restrict__ bulk_in, uint8_t* __restrict__ bulk_out, const unsigned* __restrict__ list,
         const unsigned* __restrict__ count, R tshift, int tiles_x, int tiles_y, int zc) {
  constexpr int HX = TX + 2, HY = TY + 2, HC = HX * HY;
  __shared__ R ring[4][N][HC];
  const unsigned nb = (unsigned)tiles_x * (unsigned)tiles_y * (unsigned)((p.n[2] + zc - 1) / zc);
  const unsigned cnt = min(*count, nb);
  // gridDim.x is a multiple of 8: XCD k (blocks b = k mod 8) takes part k of the list
  const unsigned g8 = gridDim.x / 8u, k = blockIdx.x % 8u;
  const unsigned hi = (unsigned)(((unsigned long long)cnt * (k + 1u)) / 8u);
  for (unsigned w = (unsigned)(((unsigned long long)cnt * k) / 8u) + blockIdx.x / 8u; w < hi; w += g8) {
    const unsigned lb = list[w];
    // entries are tile indices (the list starts zeroed); the check keeps a
    // count that disagrees with the list inside the grid (uniform per block)
    if (lb >= nb) continue;
    const Tile T = tile_at(lb, tiles_x, tiles_y, TX, TY, zc, p.n[2], D);
    phi_walk<D, N, NC, R, TX, TY, false>(p, phi, mu, phi_out, bulk_in[T.lb] != 0, bulk_out, nullptr, tshift, T,
                                         ring);
  }
}

// ---------------------------------------------------------------------------
// Chemical potential + LBM, z-marching.  Each thread walks its (x, y) column
// along z: phi^{n+1}, mu^n and U_z^{n-1} of the planes z-1, z, z+1 at its own
// column stay in registers (one new plane is loaded per step), and the
// in-plane neighbours (x +- 1, y +- 1) of phi^{n+1}, mu^n, U_x, U_y come from
// a double-buffered LDS tile: each thread writes its own column's values from
// registers, and the threads on the tile's edge also the halo cell beyond
// them (corners are never read).  The next plane's values are fetched into
// registers before a plane is computed, so their loads overlap it; one
// barrier per plane.  Threads past the grid's edge hold the wrapped (periodic)
// or clamped (wall) column, which only serves as a neighbour.
// A tile row is one 64-lane wave, so a wave's row y and plane z are uniform:
// every address is a scalar row offset plus the lane's column.
// ---------------------------------------------------------------------------
template <int D, int Q, int N, int NC, class R, int TX, int TY, bool SH, bool MT>
__global__ void __launch_bounds__(TX * TY)
k_mulbm_z(KP<R> p, const R* __restrict__ phi0, const R* __restrict__ phi1,
          const R* __restrict__ mu, const R* __restrict__ uold, const R* __restrict__ fin,
          R* __restrict__ mu_out, R* __restrict__ u_out, R* __restrict__ fout, R* __restrict__ dr_out,
          const uint8_t* __restrict__ phi_bulk, int zc_phi, R tshift, int tiles_x, int tiles_y, int zc,
          unsigned* __restrict__ todo_count) {
  static_assert(TX == 64, "one tile row per 64-lane wave");
  static_assert(TY >= 2, "edge threads own one row and one column halo cell at most");
  constexpr int HX = TX + 2, HY = TY + 2, HC = HX * HY;
  constexpr int NV = N + NC + 2;  // phi^{n+1}, mu^n, U_x, U_y per tile cell
  constexpr int NB = (D == 3) ? 2 : 1;
  __shared__ R sh[NB][NV][HC];
  const Tile T = tile_of(tiles_x, tiles_y, TX, TY, zc, p.n[2], D);
  const int tid = threadIdx.x;
  // the step's k_phi_zl, which read the list length, has finished: clear it
  // for the next step's k_phi_todo
  if (todo_count && blockIdx.x == 0 && tid == 0) atomicExch(todo_count, 0u);
  const int lx = tid % TX, ly = __builtin_amdgcn_readfirstlane(tid / TX);
  const int x = T.x0 + lx, y = T.y0 + ly;
  const bool own = x < p.n[0] && y < p.n[1];
  const int c0 = (ly + 1) * HX + (lx + 1);
  const int xw = wrap_or_clamp(x, p.n[0], p.per[0]), yw = wrap_or_clamp(y, p.n[1], p.per[1]);
  const int64_t rowc = (int64_t)yw * p.sy;  // + xw: the thread's column
  // halo cells: 0 the row halo (y0 - 1 or y0 + TY), 1 the column halo (x0 - 1 or x0 + TX)
  const bool hrow = ly == 0 || ly == TY - 1, hcol = lx == 0 || lx == TX - 1;
  const int hy = (ly == 0) ? -1 : TY, hx = (lx == 0) ? -1 : TX;
  const int hi0 = (hy + 1) * HX + (lx + 1), hi1 = (ly + 1) * HX + (hx + 1);
  const int64_t hrow0 = (int64_t)wrap_or_clamp(T.y0 + hy, p.n[1], p.per[1]) * p.sy;  // + xw
  const int hx1 = wrap_or_clamp(T.x0 + hx, p.n[0], p.per[0]);                        // + rowc
  const PullX px = pull_x(x, p.n[0], p.per[0]);
  // phi_bulk (k_phi_z's flags of this step, null when there are none): where
  // the k_phi_z block holding this tile and these planes left every cell bulk,
  // phi^n = phi^{n+1} there, so phi^n is not read (the two-phase, one-solute
  // instances, where that saves a phase field per cell at no register cost)
  constexpr bool SKIP0 = !SH && !MT && N == 2 && NC == 1;
  bool same0 = false;
  if constexpr (SKIP0) {
    if (phi_bulk) {
      const unsigned tz = (D == 3) ? (unsigned)(T.z0 / zc_phi) : 0u;
      const unsigned t0 = T.lb % (unsigned)(tiles_x * tiles_y);
      same0 = phi_bulk[t0 + (unsigned)(tiles_x * tiles_y) * tz] != 0;
    }
  }
  auto zoff = [&](int zz) -> int64_t {
    return (D == 3) ? (int64_t)wrap_or_clamp(zz, p.n[2], p.per[2]) * p.sz : 0;
  };

  // own column, planes z-1 (index 0), z (1), z+1 (2)
  R cph[3][N], cmu[3][NC], cuz[3];
  auto fetch_col = [&](int zz, R (&ph)[N], R (&m)[NC], R& uz) {
    const int64_t j = zoff(zz) + rowc;
#pragma unroll
    for (int q = 0; q < N; ++q) ph[q] = *lane_at(phi1, q * p.cells + j, xw);
#pragma unroll
    for (int q = 0; q < NC; ++q) m[q] = *lane_at(mu, q * p.cells + j, xw);
    uz = (D == 3) ? *lane_at(uold, (D - 1) * p.cells + j, xw) : R(0);
  };
  // values of one plane that go to LDS besides the column's phi and mu: own
  // U_x, U_y and the halo cells
  R cuxy[2], hv[2][NV], ph0[N];
  auto fetch_plane = [&](int zz) {
    const int64_t zo = zoff(zz);
    cuxy[0] = *lane_at(uold, zo + rowc, xw);
    cuxy[1] = *lane_at(uold, p.cells + zo + rowc, xw);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (h == 0 ? hrow : hcol) {
        const int64_t j = zo + (h == 0 ? hrow0 : rowc);
        const int l = (h == 0) ? xw : hx1;
#pragma unroll
        for (int q = 0; q < N; ++q) hv[h][q] = *lane_at(phi1, q * p.cells + j, l);
#pragma unroll
        for (int q = 0; q < NC; ++q) hv[h][N + q] = *lane_at(mu, q * p.cells + j, l);
        hv[h][N + NC] = *lane_at(uold, j, l);
        hv[h][N + NC + 1] = *lane_at(uold, p.cells + j, l);
      }
    }
  };
  auto write_plane = [&](int bf) {
#pragma unroll
    for (int q = 0; q < N; ++q) sh[bf][q][c0] = cph[1][q];
#pragma unroll
    for (int q = 0; q < NC; ++q) sh[bf][N + q][c0] = cmu[1][q];
    sh[bf][N + NC][c0] = cuxy[0];
    sh[bf][N + NC + 1][c0] = cuxy[1];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      if (hrow) sh[bf][v][hi0] = hv[0][v];
      if (hcol) sh[bf][v][hi1] = hv[1][v];
    }
  };
  auto fetch_ph0 = [&](int zz, R (&o)[N]) {
    if (same0) return;
    const int64_t j = zoff(zz) + rowc;
#pragma unroll
    for (int q = 0; q < N; ++q) o[q] = *lane_at(phi0, q * p.cells + j, xw);
  };

  if (D == 3) {
    fetch_col(T.z0 - 1, cph[0], cmu[0], cuz[0]);
    fetch_col(T.z0 + 1, cph[2], cmu[2], cuz[2]);
  }
  fetch_col(T.z0, cph[1], cmu[1], cuz[1]);
  fetch_plane(T.z0);
  fetch_ph0(T.z0, ph0);
  {
    // every value loaded before the loop is consumed here, so none is still
    // in flight when the loop starts: the loop's own prefetch is then waited
    // for where the next plane uses it, not (as the compiler's wait counting
    // would otherwise place it, merging the loop's entry with its back edge)
    // at the first use of a value carried into the loop, in mid-plane
    auto settle = [](R& v) { asm volatile("" : "+v"(v)); };
#pragma unroll
    for (int k = 0; k < 3; ++k) {
#pragma unroll
      for (int q = 0; q < N; ++q) settle(cph[k][q]);
#pragma unroll
      for (int q = 0; q < NC; ++q) settle(cmu[k][q]);
      settle(cuz[k]);
    }
#pragma unroll
    for (int q = 0; q < N; ++q) settle(ph0[q]);
    settle(cuxy[0]);
    settle(cuxy[1]);
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int v = 0; v < NV; ++v) settle(hv[h][v]);
  }
  for (int z = T.z0; z < T.z1; ++z) {
    const int bf = (z - T.z0) & (NB - 1);
    write_plane(bf);
    __syncthreads();
    // next plane's loads, in flight while this plane is computed
    R nph[N] = {}, nmu[NC] = {}, nuz = R(0), np0[N] = {};
    if (z + 1 < T.z1) {
      fetch_plane(z + 1);
      fetch_ph0(z + 1, np0);
      if (D == 3) fetch_col(z + 2, nph, nmu, nuz);
    }
    if (own) {
      // strides and coordinates opaque per plane: addresses and the other
      // quantities of the cell are formed anew on every plane instead of being
      // carried along z (as pointers, one scalar register pair per buffer and
      // population, or as per-lane values held in vector registers)
      KP<R> q = p;
      int xq = x, yq = y;
      asm volatile("" : "+s"(q.cells), "+s"(q.sy), "+s"(q.sz), "+v"(xq), "+s"(yq));
      R ph1n[2 * D + 1][N], mun[2 * D + 1][NC], uc[D], un[D][2];
      const int off[4] = {-1, 1, -HX, HX};
#pragma unroll
      for (int q = 0; q < N; ++q) {
        ph1n[0][q] = cph[1][q];
#pragma unroll
        for (int j = 0; j < 4; ++j) ph1n[1 + j][q] = sh[bf][q][c0 + off[j]];
        if (D == 3) {
          ph1n[2 * D - 1][q] = cph[0][q];
          ph1n[2 * D][q] = cph[2][q];
        }
      }
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        mun[0][q] = cmu[1][q];
#pragma unroll
        for (int j = 0; j < 4; ++j) mun[1 + j][q] = sh[bf][N + q][c0 + off[j]];
        if (D == 3) {
          mun[2 * D - 1][q] = cmu[0][q];
          mun[2 * D][q] = cmu[2][q];
        }
      }
      uc[0] = sh[bf][N + NC][c0];
      uc[1] = sh[bf][N + NC + 1][c0];
      un[0][0] = sh[bf][N + NC][c0 - 1];
      un[0][1] = sh[bf][N + NC][c0 + 1];
      un[1][0] = sh[bf][N + NC + 1][c0 - HX];
      un[1][1] = sh[bf][N + NC + 1][c0 + HX];
      if (D == 3) {
        uc[D - 1] = cuz[1];
        un[D - 1][0] = cuz[0];
        un[D - 1][1] = cuz[2];
      }
      R p0[N];
#pragma unroll
      for (int k = 0; k < N; ++k) p0[k] = same0 ? cph[1][k] : ph0[k];
      mulbm_core<D, Q, N, NC, R, SH, MT>(q, xq, yq, z, px, tshift, ph1n, mun, uc, un, p0, fin, mu_out, u_out,
                                         fout, dr_out);
    }
#pragma unroll
    for (int q = 0; q < N; ++q) {
      cph[0][q] = cph[1][q];
      cph[1][q] = cph[2][q];
      cph[2][q] = nph[q];
      ph0[q] = np0[q];
    }
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      cmu[0][q] = cmu[1][q];
      cmu[1][q] = cmu[2][q];
      cmu[2][q] = nmu[q];
    }
    cuz[0] = cuz[1];
    cuz[1] = cuz[2];
    cuz[2] = nuz;
  }
}

// ---------------------------------------------------------------------------
// Auxiliary kernels (read, write, totals, health).  One thread per cell on a
// 1D grid.
// ---------------------------------------------------------------------------

// Moving frame (Case 2 follows the growth front with a moving frame; the
// paper gives no details, the reading is stated with the host code).
// k_front: the largest pull-axis index of a cell whose liquid fraction is at
// most 1/2 (-1 if none), max-reduced over each wave, then one atomic per wave.
template <int N, class R>
__global__ void __launch_bounds__(256) k_front(KP<R> p, const R* __restrict__ phi, int* __restrict__ front) {
  const int64_t P = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int v = -1;
  if (P < p.cells && phi[(N - 1) * p.cells + P] <= R(0.5)) {
    const int64_t c = (p.pull_axis == 0) ? P % p.n[0]
                      : (p.pull_axis == 1) ? (P / p.sy) % p.n[1] : P / p.sz;
    v = (int)c;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
  if ((threadIdx.x & 63) == 0 && v >= 0) atomicMax(front, v);
}

// k_shift: out = in moved down an axis by d cells (index stride `stride`,
// extent n_ax); the last d planes repeat the last plane of `in`.
template <class R>
__global__ void k_shift(const R* __restrict__ in, R* __restrict__ out, int64_t count, int64_t cells,
                        int64_t stride, int64_t n_ax, int64_t d) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int64_t P = i % cells;
  const int64_t c = (P / stride) % n_ax;
  const int64_t src = min(c + d, n_ax - 1);
  out[i] = in[i + (src - c) * stride];
}

// f^n_k(P) = stored f*_k(P - c_k) (+ bounce-back), plus w_k rho0: the full f.
template <int D, int Q, class R>
__global__ void k_gather_f(KP<R> p, const R* __restrict__ fin, double* __restrict__ out) {
  using L = Lat<Q>;
  const int64_t P = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (P >= p.cells) return;
  const int x = (int)(P % p.n[0]);
  const int y = (int)((P / p.sy) % p.n[1]);
  const int z = (int)(P / p.sz);
  for (int k = 0; k < L::Q; ++k)
    out[k * p.cells + P] = (double)pull_f<D, Q, R>(p, fin, x, y, z, P, k) + L::w(k) * (double)p.rho0;
}

// inverse of k_gather_f: the stored pre-streaming f* that streams to f^n.
// With d > 0 it inverts the pull of f^n moved down axis `ax` by d cells (the
// moving frame): every read of f^n at coordinate c along ax reads c + d,
// clamped to the last plane.
template <int D, int Q, class R>
__global__ void k_scatter_f(KP<R> p, const double* __restrict__ fn, R* __restrict__ fst, int ax, int d) {
  using L = Lat<Q>;
  const int64_t Qc = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (Qc >= p.cells) return;
  const int x = (int)(Qc % p.n[0]);
  const int y = (int)((Qc / p.sy) % p.n[1]);
  const int z = (int)(Qc / p.sz);
  auto at = [&](int c0, int c1, int c2) -> int64_t {
    int c[3] = {c0, c1, c2};
    c[ax] = min(c[ax] + d, p.n[ax] - 1);
    return (int64_t)c[2] * p.sz + (int64_t)c[1] * p.sy + c[0];
  };
  for (int k = 0; k < L::Q; ++k) {
    int dst[3] = {x + L::c(k, 0), y + L::c(k, 1), z + L::c(k, 2)};
    bool in = true;
    for (int a = 0; a < D; ++a)
      if (dst[a] < 0 || dst[a] >= p.n[a]) {
        if (p.per[a])
          dst[a] = (dst[a] + p.n[a]) % p.n[a];
        else
          in = false;
      }
    double val;
    if (in) {
      val = fn[k * p.cells + at(dst[0], dst[1], dst[2])] - L::w(k) * (double)p.rho0;
    } else {
      const int kb = L::opp(k);
      val = fn[kb * p.cells + at(x, y, z)] - L::w(kb) * (double)p.rho0;
      if (L::c(kb, 1) < 0 && !p.per[1] && y - L::c(kb, 1) >= p.n[1])
        val -= 6.0 * L::w(kb) * (double)p.rho0 * L::c(kb, 0) * (double)p.lid_u;
    }
    fst[k * p.cells + Qc] = (R)val;
  }
}

template <class R>
__global__ void k_to_double(const R* __restrict__ in, double* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (double)in[i];
}

template <class R>
__global__ void k_from_double(const double* __restrict__ in, R* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (R)in[i];
}

// chemical potentials: FP64 mu <-> stored mu - mu_ref, component i = idx / cells
template <class R>
__global__ void k_mu_to_double(const R* __restrict__ in, double* __restrict__ out, int64_t cells,
                               int nc, double r0, double r1) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nc * cells) out[i] = (double)in[i] + (i < cells ? r0 : r1);
}
template <class R>
__global__ void k_mu_from_double(const double* __restrict__ in, R* __restrict__ out, int64_t cells,
                                 int nc, double r0, double r1) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nc * cells) out[i] = (R)(in[i] - (i < cells ? r0 : r1));
}
template <class R>
__global__ void k_mu_native(const R* __restrict__ in, R* __restrict__ out, int64_t cells, int nc,
                            R r0, R r1) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nc * cells) out[i] = in[i] + (i < cells ? r0 : r1);
}

// derived per-cell fields in FP64: 0 rho, 1 mixture composition C (nc comps),
// 2 temperature, 3 active-set bitmask
template <int D, int Q, int N, int NC, class R>
__global__ void k_derived(KP<R> p, int which, const R* __restrict__ phi, const R* __restrict__ mu,
                          const double* __restrict__ fgathered, double tshift_d,
                          double* __restrict__ out) {
  using L = Lat<Q>;
  const int64_t P = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (P >= p.cells) return;
  const int x = (int)(P % p.n[0]);
  const int y = (int)((P / p.sy) % p.n[1]);
  const int z = (int)(P / p.sz);
  if (which == 0) {
    double r = 0.0;
    for (int k = 0; k < L::Q; ++k) r += fgathered[k * p.cells + P];
    out[P] = r;
  } else if (which == 1) {
    double ph[N], h[N], m[NC];
    for (int b = 0; b < N; ++b) ph[b] = (double)phi[b * p.cells + P];
    for (int i = 0; i < NC; ++i) m[i] = (double)mu[i * p.cells + P];
    interp_h<N, double>(ph, h);
    const int pos[3] = {x, y, z};
    const double td = (p.G != R(0)) ? (double)p.G * ((double)pos[p.pull_axis] - tshift_d) : (double)p.tdev_iso;
    for (int i = 0; i < NC; ++i) {
      double c = 0.0;
      for (int b = 0; b < N; ++b) {
        double C = p.c0s_d[b][i] + (double)p.mT[b][i] * td;
        for (int k = 0; k < NC; ++k) C += (double)p.chi[i][k] * m[k];
        c += h[b] * C;
      }
      out[i * p.cells + P] = c;
    }
  } else if (which == 2) {
    const int pos[3] = {x, y, z};
    out[P] = (double)p.T_E + ((p.G != R(0)) ? (double)p.G * ((double)pos[p.pull_axis] - tshift_d)
                                              : (double)p.tdev_iso);
  } else {
    unsigned mask = 0u;
    for (int k = 0; k < L::Q; ++k) {
      const int xx = nb_field(x, L::c(k, 0), p.n[0], p.per[0]);
      const int yy = nb_field(y, L::c(k, 1), p.n[1], p.per[1]);
      const int zz = (D == 3) ? nb_field(z, L::c(k, 2), p.n[2], p.per[2]) : 0;
      const int64_t j = (int64_t)zz * p.sz + (int64_t)yy * p.sy + xx;
      for (int b = 0; b < N; ++b)
        if (phi[b * p.cells + j] > R(0)) mask |= 1u << b;
    }
    out[P] = (double)mask;
  }
}

// FP64 block partial sums in a fixed order: solute (NC values, which 0),
// mass (which 1) or the loss 1/2 sum_a (phi_a - target_a)^2 (which 2).
constexpr int RED_BLOCK = 256;
template <int D, int Q, int N, int NC, class R>
__global__ void __launch_bounds__(RED_BLOCK)
k_partial(KP<R> p, int which, const R* __restrict__ phi, const R* __restrict__ mu,
          const R* __restrict__ f, const double* __restrict__ target, double tshift_d,
          double* __restrict__ partial) {
  using L = Lat<Q>;
  __shared__ double sh[NC][RED_BLOCK];
  const int t = threadIdx.x;
  double acc[NC];
  for (int i = 0; i < NC; ++i) acc[i] = 0.0;
  for (int64_t P = (int64_t)blockIdx.x * RED_BLOCK + t; P < p.cells;
       P += (int64_t)gridDim.x * RED_BLOCK) {
    if (which == 0) {
      double ph[N], h[N], m[NC];
      for (int b = 0; b < N; ++b) ph[b] = (double)phi[b * p.cells + P];
      for (int i = 0; i < NC; ++i) m[i] = (double)mu[i * p.cells + P];
      interp_h<N, double>(ph, h);
      const int pos[3] = {(int)(P % p.n[0]), (int)((P / p.sy) % p.n[1]), (int)(P / p.sz)};
      const double td = (p.G != R(0)) ? (double)p.G * ((double)pos[p.pull_axis] - tshift_d) : (double)p.tdev_iso;
      for (int i = 0; i < NC; ++i) {
        double c = 0.0;
        for (int b = 0; b < N; ++b) {
          double C = p.c0s_d[b][i] + (double)p.mT[b][i] * td;
          for (int k = 0; k < NC; ++k) C += (double)p.chi[i][k] * m[k];
          c += h[b] * C;
        }
        acc[i] += c;
      }
    } else if (which == 1) {
      const int x = (int)(P % p.n[0]);
      const int y = (int)((P / p.sy) % p.n[1]);
      const int z = (int)(P / p.sz);
      double r = 0.0;
      for (int k = 0; k < L::Q; ++k)
        r += (double)pull_f<D, Q, R>(p, f, x, y, z, P, k) + L::w(k) * (double)p.rho0;
      acc[0] += r;
    } else {
      double r = 0.0;
      for (int b = 0; b < N; ++b) {
        const double d = (double)phi[b * p.cells + P] - target[b * p.cells + P];
        r += d * d;
      }
      acc[0] += 0.5 * r;
    }
  }
  for (int i = 0; i < NC; ++i) sh[i][t] = acc[i];
  __syncthreads();
  for (int s = RED_BLOCK / 2; s > 0; s >>= 1) {
    if (t < s)
      for (int i = 0; i < NC; ++i) sh[i][t] += sh[i][t + s];
    __syncthreads();
  }
  // one value per block and component of this total, in the stride
  // k_final_sum reads: NC for the solute, 1 for the mass and the loss
  const int ncomp = (which == 0) ? NC : 1;
  if (t == 0)
    for (int i = 0; i < ncomp; ++i) partial[blockIdx.x * ncomp + i] = sh[i][0];
}

__global__ void k_final_sum(const double* __restrict__ partial, int nblocks, int ncomp,
                            double* __restrict__ out) {
  __shared__ double sh[RED_BLOCK];
  for (int i = 0; i < ncomp; ++i) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += RED_BLOCK) acc += partial[b * ncomp + i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = RED_BLOCK / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[i] = sh[0];
    __syncthreads();
  }
}

// dL/dphi of the loss 1/2 sum (phi - target)^2: phi - target in FP64
template <class R>
__global__ void k_loss_seed(const R* __restrict__ phi, const double* __restrict__ target,
                            double* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (double)phi[i] - target[i];
}

// ---------------------------------------------------------------------------
// Bandwidth probes (measurement only): the memory access patterns of the
// population update without its arithmetic, on 19 FP32 arrays of an
// n0 x n1 x n2 grid (all axes periodic).  k_probe_copy19: out_k(P) = in_k(P);
// k_probe_pull19: out_k(P) = in_k(P - c_k) with the D3Q19 velocities, one
// thread per cell in 256-cell blocks; k_probe_pull19_z: the same pull in the
// launch shape of k_mulbm_z (64 x TY tiles walking ZC planes, XCD-aware tile
// order).  Streaming (nontemporal) loads and stores as in the step kernels.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_probe_copy19(const float* __restrict__ in, float* __restrict__ out,
                                                      int64_t cells) {
  const int64_t P = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (P >= cells) return;
#pragma unroll
  for (int k = 0; k < 19; ++k)
    __builtin_nontemporal_store(__builtin_nontemporal_load(&in[k * cells + P]), &out[k * cells + P]);
}

__device__ __forceinline__ void probe_pull_cell(const float* __restrict__ in, float* __restrict__ out, int x, int y,
                                                int z, int n0, int n1, int n2, int64_t cells) {
  using L = Lat<19>;
  const int64_t P = ((int64_t)z * n1 + y) * n0 + x;
  float v[19];
#pragma unroll
  for (int k = 0; k < 19; ++k) {
    const int xs = (x - L::c(k, 0) + n0) % n0, ys = (y - L::c(k, 1) + n1) % n1, zs = (z - L::c(k, 2) + n2) % n2;
    v[k] = __builtin_nontemporal_load(&in[k * cells + ((int64_t)zs * n1 + ys) * n0 + xs]);
  }
#pragma unroll
  for (int k = 0; k < 19; ++k) __builtin_nontemporal_store(v[k], &out[k * cells + P]);
}

__global__ void __launch_bounds__(256) k_probe_pull19(const float* __restrict__ in, float* __restrict__ out, int n0,
                                                      int n1, int n2) {
  const int64_t cells = (int64_t)n0 * n1 * n2;
  const int64_t P = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (P >= cells) return;
  probe_pull_cell(in, out, (int)(P % n0), (int)((P / n0) % n1), (int)(P / ((int64_t)n0 * n1)), n0, n1, n2, cells);
}

template <int TY>
__global__ void __launch_bounds__(64 * TY) k_probe_pull19_z(const float* __restrict__ in, float* __restrict__ out,
                                                            int n0, int n1, int n2, int zc) {
  const int64_t cells = (int64_t)n0 * n1 * n2;
  const Tile T = tile_of(n0 / 64, n1 / TY, 64, TY, zc, n2, 3);
  const int x = T.x0 + (int)threadIdx.x % 64, y = T.y0 + (int)threadIdx.x / 64;
  for (int z = T.z0; z < T.z1; ++z) probe_pull_cell(in, out, x, y, z, n0, n1, n2, cells);
}

// health: NaN/Inf in phi or mu, or rho <= 0, records the smallest step seen
template <int D, int Q, int N, int NC, class R>
__global__ void k_health(KP<R> p, const R* __restrict__ phi, const R* __restrict__ mu,
                         const R* __restrict__ f, unsigned long long step,
                         unsigned long long* __restrict__ bad_step) {
  using L = Lat<Q>;
  const int64_t P = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (P >= p.cells) return;
  const int x = (int)(P % p.n[0]);
  const int y = (int)((P / p.sy) % p.n[1]);
  const int z = (int)(P / p.sz);
  bool bad = false;
  for (int b = 0; b < N; ++b) bad |= !isfinite(phi[b * p.cells + P]);
  for (int i = 0; i < NC; ++i) bad |= !isfinite(mu[i * p.cells + P]);
  R r = p.rho0;
  for (int k = 0; k < L::Q; ++k) r += pull_f<D, Q, R>(p, f, x, y, z, P, k);
  bad |= !(r > R(0));
  if (bad) atomicMin(bad_step, step);
}

}  // namespace gpf
