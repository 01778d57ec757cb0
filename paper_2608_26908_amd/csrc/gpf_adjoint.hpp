// gpf_adjoint.hpp -- discrete adjoint of one coupled step (reverse mode of
// the forward kernels, written by hand) and the FP64 parameter gradients.
//
// State at step n: X^n = (phi^n, mu^n, U^{n-1}, f^n), f^n the populations
// after streaming (held on the device as the previous post-collision f*,
// pulled on use).  One reverse step maps the adjoint of X^{n+1} to the adjoint
// of X^n, reading X^n and X^{n+1} from the recomputed tape:
//   k_adj_lbm   streaming transpose + collision VJP, then   -> lam f^n, lam phi_l' (partial), d gbeta,
//               w = chi_tot^{-1} lam mu'                        w, lam mu^n (direct term)
//   k_adj_muphi faces of the mu update (gather), then the   -> lam mu^n, lam U^{n-1}, lam phi^n, d D,
//               projection and local phase-field terms         Rbar, d tau
//   k_adj_vjp   reverse of each face flux / cell term, once  -> their adjoint values, d delta
//   k_adj_phi2  gather of the contributions they imply      -> lam phi^n
// k_adj_lbm of step n - 1 does not read lam phi^n, so k_adj_phi2_lbm runs it
// in the same launch as the gather of step n (used on small grids).
// Every kernel gathers into the cells it owns: no atomics, deterministic.
// Parameter derivatives are reduced per block in FP64 and summed in a fixed
// order.  Hessian-vector products of the gradient energy come from forward
// mode through dAdq.
#pragma once
#include "gpf_kernels.hpp"

namespace gpf {

enum { G_DELTA = 0, G_TAU = 1, G_D0 = 2, G_D1 = 3, G_GB0 = 4, G_GB1 = 5, NG = 6 };
constexpr int ADJ_BLOCK = 256;

// Cell of a thread.  Work-groups are dealt to the 8 XCDs round-robin
// (work-group b runs on XCD b mod 8); the grid is laid out so that XCD k owns
// the rows [k ny / 8, (k + 1) ny / 8) of every plane and walks them plane by
// plane.  A cell's neighbours in y and z are then, except at a slab edge,
// read through the same L2, while all eight XCDs stream through the same
// planes.  False for the padding slots at the end of an XCD's range.  blk:
// the work-group's index within a grid of the linear layout (a launch that
// runs several such grids side by side passes blockIdx.x minus the offset of
// its grid, a multiple of 8).
__device__ __forceinline__ bool adj_cell(const int (&n)[3], int64_t sy, int64_t sz, int64_t& P, int& x,
                                         int& y, int& z, unsigned blk = blockIdx.x) {
  const unsigned k = blk % 8u, i = blk / 8u;
  const int y0 = (int)(((int64_t)k * n[1]) / 8);
  const unsigned h = (unsigned)((int)(((int64_t)(k + 1) * n[1]) / 8) - y0);
  const unsigned s = i * (unsigned)ADJ_BLOCK + threadIdx.x;
  if (s >= (unsigned)n[0] * h * (unsigned)n[2]) return false;
  x = (int)(s % (unsigned)n[0]);
  const unsigned r = s / (unsigned)n[0];
  y = y0 + (int)(r % h);
  z = (int)(r / h);
  P = (int64_t)z * sz + (int64_t)y * sy + x;
  return true;
}

// Per-block FP64 partial sums of the NG parameter derivatives, in a fixed
// order (shuffle tree within each wave, then the waves in turn), added to the
// block's running sums over the reverse sweep: every block owns its slots, so
// no atomics are needed and the result is deterministic.
__device__ __forceinline__ void block_partials(double (&g)[NG], double* __restrict__ part,
                                               unsigned slot = blockIdx.x) {
  constexpr int NW = ADJ_BLOCK / 64;
  __shared__ double sh[NG][NW];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
#pragma unroll
  for (int i = 0; i < NG; ++i) {
    double v = g[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) sh[i][wv] = v;
  }
  __syncthreads();
  if (t < NG) {
    double s = sh[t][0];
#pragma unroll
    for (int w = 1; w < NW; ++w) s += sh[t][w];
    part[(int64_t)slot * NG + t] += s;
  }
}

// phi^n neighbourhood of a cell, walls mirrored, periodic axes wrapped
template <int D, int N, class R>
__device__ __forceinline__ void load_stencil(const KP<R>& p, const R* __restrict__ phi, int x, int y,
                                             int z, R (&v)[N][3][3][3]) {
#pragma unroll
  for (int dz = (D == 3 ? -1 : 0); dz <= (D == 3 ? 1 : 0); ++dz)
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        if (dx != 0 && dy != 0 && dz != 0) continue;
        const int xx = nb_field(x, dx, p.n[0], p.per[0]);
        const int yy = nb_field(y, dy, p.n[1], p.per[1]);
        const int zz = (D == 3) ? nb_field(z, dz, p.n[2], p.per[2]) : 0;
        const int64_t j = (int64_t)zz * p.sz + (int64_t)yy * p.sy + xx;
#pragma unroll
        for (int b = 0; b < N; ++b) v[b][dz + 1][dy + 1][dx + 1] = phi[b * p.cells + j];
      }
}

// d^2 h_b / dphi_a dphi_g.  For N >= 3, with h_b's extra term 2 phi_b e_b:
// 2 (delta_ab de_b/dphi_g + delta_gb de_b/dphi_a + phi_b d2e_b/dphi_a dphi_g),
// de_b/dphi_g = sum of the phases other than b and g (g != b), and
// d2e_b/dphi_a dphi_g = 1 for distinct a, g, b.
template <int N, class R>
__device__ __forceinline__ R d2h(const R (&ph)[N], int b, int a, int g) {
  R r = (a == b && g == b) ? R(6) - R(12) * ph[b] : R(0);
  if constexpr (N == 3) {
    if (a != g) r += R(2) * ph[3 - a - g];
  } else if constexpr (N >= 4) {
    if (a != g) {
      if (a == b || g == b) {
        const int o = (a == b) ? g : a;
        R rest = R(0);
#pragma unroll
        for (int k = 0; k < N; ++k)
          if (k != b && k != o) rest += ph[k];
        r += R(2) * rest;
      } else {
        r += R(2) * ph[b];
      }
    }
  }
  return r;
}

// ---------------------------------------------------------------------------
// 1. streaming transpose + collision VJP
// ---------------------------------------------------------------------------
// The collision depends on the pulled populations only through rho and U.
// TAPE: rho - rho0 of the step was stored by the forward recomputation and U
// is the step's own output, so f is not read; otherwise both are recomputed
// from the pulled f (the last step of a checkpoint segment).
template <int D, int Q, int N, int NC, class R, bool TAPE>
__device__ __forceinline__ void adj_lbm_cell(const KP<R>& p, const int64_t P, const int x, const int y,
                                             const int z, const R* __restrict__ fst,
                                             const R* __restrict__ dr_t, const R* __restrict__ u1,
                                             const R* __restrict__ phi1, const R* __restrict__ mu1,
                                             const R* __restrict__ lf1, const R* __restrict__ lu1,
                                             const R* __restrict__ lmu1, R* __restrict__ lf0,
                                             R* __restrict__ t_phil, R* __restrict__ w,
                                             R* __restrict__ lmu0, R tshift1, double (&gpart)[NG]) {
  using L = Lat<Q>;
  {
    R f[TAPE ? 1 : L::Q], ob[L::Q];
    // offset of the cell one step along -e_a (index 0) and +e_a (index 1) from
    // P, wrapped on a periodic axis, and whether that cell lies behind a wall
    const int pos[3] = {x, y, z};
    const int64_t stride[3] = {1, p.sy, p.sz};
    int64_t off[3][2];
    bool wall[3][2];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int si = 0; si < 2; ++si) {
        const int t = pos[a] + (si ? 1 : -1);
        wall[a][si] = a < D && !p.per[a] && (t < 0 || t >= p.n[a]);
        const int w = (t < 0) ? t + p.n[a] : (t >= p.n[a] ? t - p.n[a] : t);
        off[a][si] = (a < D) ? (int64_t)(w - pos[a]) * stride[a] : 0;
      }
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
      if constexpr (!TAPE) f[k] = pull_f<D, Q, R>(p, fst, x, y, z, P, k);
      // f*_k(P) streams to f_k(P + c_k), or is reflected into f_{opp k}(P)
      int64_t dst = P;
      bool in = true;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        if (L::c(k, a) == 0) continue;
        const int si = L::c(k, a) > 0 ? 1 : 0;
        dst += off[a][si];
        in = in && !wall[a][si];
      }
      // every adjoint population is read once per reverse step: a streaming load
      ob[k] = __builtin_nontemporal_load(in ? &lf1[k * p.cells + dst] : &lf1[L::opp(k) * p.cells + P]);
    }
    const R phil = phi1[(N - 1) * p.cells + P];
    R mu[NC];
#pragma unroll
    for (int i = 0; i < NC; ++i) mu[i] = mu1[i * p.cells + P];
    // ---- forward recomputation ----
    R dr = R(0), mom[D];
#pragma unroll
    for (int a = 0; a < D; ++a) mom[a] = R(0);
    if constexpr (TAPE) {
      dr = dr_t[P];
    } else {
#pragma unroll
      for (int k = 0; k < L::Q; ++k) {
        dr += f[k];
#pragma unroll
        for (int a = 0; a < D; ++a)
          if (L::c(k, a) != 0) mom[a] += R(L::c(k, a)) * f[k];
      }
    }
    const R rho = p.rho0 + dr;
    // the liquid's composition at the step's new temperature T^{n+1}
    const R td1 = tdev_at(p, pos[p.pull_axis], tshift1);
    R Cl[NC], bsum = R(0);
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      Cl[i] = p.c0s[N - 1][i] + p.mT[N - 1][i] * td1;
#pragma unroll
      for (int k = 0; k < NC; ++k) Cl[i] += p.chi[i][k] * mu[k];
      bsum += p.gbeta[i] * (Cl[i] - p.c_ref[i]);
    }
    const int ga = p.grav_axis;
    R FB[D];
#pragma unroll
    for (int a = 0; a < D; ++a) FB[a] = R(0);
    FB[ga] = -rho * phil * bsum * p.grav_sign;
    const R sol = (R(1) - phil) * (R(1) - phil);
    const R den = rho * (R(1) + R(0.5) * p.kappa * sol);
    const bool moving = phil != R(0);
    const R iden = moving ? R(1) / den : R(0);
    R u[D], F[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      if constexpr (TAPE)
        u[a] = u1[a * p.cells + P];
      else
        u[a] = (mom[a] + R(0.5) * FB[a]) * iden;
      F[a] = FB[a] - p.kappa * rho * sol * u[a];
    }
    R uu = R(0);
#pragma unroll
    for (int a = 0; a < D; ++a) uu += u[a] * u[a];
    const R pref = p.guo;
    const R keep = R(1) - p.omega;
    // ---- reverse ----
    R fb[L::Q], drb = R(0), rhob = R(0), uub = R(0), uFb = R(0), ub[D], Fb[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      ub[a] = lu1[a * p.cells + P];
      Fb[a] = R(0);
    }
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
      R cu = R(0), cF = R(0);
#pragma unroll
      for (int a = 0; a < D; ++a)
        if (L::c(k, a) != 0) {
          cu += R(L::c(k, a)) * u[a];
          cF += R(L::c(k, a)) * F[a];
        }
      const R wk = R(L::w(k));
      fb[k] = keep * ob[k];
      const R feqb = ob[k] * p.omega, Sb = ob[k];
      drb += wk * feqb;
      rhob += wk * feqb * (R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu);
      const R cub = wk * feqb * rho * (R(3) + R(9) * cu) + R(9) * pref * wk * Sb * cF;
      uub += -R(1.5) * wk * feqb * rho;
      const R cFb = pref * wk * Sb * (R(3) + R(9) * cu);
      uFb += -R(3) * pref * wk * Sb;
#pragma unroll
      for (int a = 0; a < D; ++a)
        if (L::c(k, a) != 0) {
          ub[a] += cub * R(L::c(k, a));
          Fb[a] += cFb * R(L::c(k, a));
        }
    }
#pragma unroll
    for (int a = 0; a < D; ++a) {
      ub[a] += R(2) * u[a] * uub + F[a] * uFb;
      Fb[a] += u[a] * uFb;
    }
    // F = FB - kappa rho sol u
    R FBb[D], solb = R(0);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      FBb[a] = Fb[a];
      rhob += -p.kappa * sol * u[a] * Fb[a];
      solb += -p.kappa * rho * u[a] * Fb[a];
      ub[a] += -p.kappa * rho * sol * Fb[a];
    }
    // u = (m + FB / 2) / den where phi_l != 0
    R mb[D], denb = R(0);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      mb[a] = ub[a] * iden;
      if (moving) {
        FBb[a] += R(0.5) * ub[a] * iden;
        denb += -ub[a] * u[a] * iden;
      }
    }
    rhob += denb * (R(1) + R(0.5) * p.kappa * sol);
    solb += denb * rho * R(0.5) * p.kappa;
    R philb = -R(2) * (R(1) - phil) * solb;
    rhob += -phil * bsum * p.grav_sign * FBb[ga];
    philb += -rho * bsum * p.grav_sign * FBb[ga];
    const R bb = -rho * phil * p.grav_sign * FBb[ga];
    R mub[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) mub[k] = R(0);
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      gpart[G_GB0 + i] = (double)((Cl[i] - p.c_ref[i]) * bb);
      const R Clb = p.gbeta[i] * bb;
#pragma unroll
      for (int k = 0; k < NC; ++k) mub[k] += p.chi[i][k] * Clb;
    }
    drb += rhob;
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
      R v = fb[k] + drb;
#pragma unroll
      for (int a = 0; a < D; ++a)
        if (L::c(k, a) != 0) v += mb[a] * R(L::c(k, a));
      __builtin_nontemporal_store(v, &lf0[k * p.cells + P]);
    }
    t_phil[P] = philb;
    // lam mu' in full, its direct pass to lam mu^n (mu' = mu + ...) and
    // w = chi_tot^{-T} lam mu' with chi_tot = sum_a h_a(phi') chi (symmetric)
    R ph[N], h[N], mt[NC];
#pragma unroll
    for (int b = 0; b < N; ++b) ph[b] = phi1[b * p.cells + P];
    interp_h<N, R>(ph, h);
    R sh = R(0);
#pragma unroll
    for (int b = 0; b < N; ++b) sh += h[b];
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      mt[i] = lmu1[i * p.cells + P] + mub[i];
      lmu0[i * p.cells + P] = mt[i];
    }
    if (NC == 1) {
      w[P] = mt[0] / (sh * p.chi[0][0]);
    } else {
      const R a11 = sh * p.chi[0][0], a12 = sh * p.chi[0][1];
      const R a21 = sh * p.chi[1][0], a22 = sh * p.chi[1][NC - 1];
      const R idet = R(1) / (a11 * a22 - a12 * a21);
      w[P] = (a22 * mt[0] - a21 * mt[NC - 1]) * idet;
      w[p.cells + P] = (-a12 * mt[0] + a11 * mt[NC - 1]) * idet;
    }
  }
}

template <int D, int Q, int N, int NC, class R, bool TAPE>
__global__ void __launch_bounds__(ADJ_BLOCK)
k_adj_lbm(KP<R> p, const R* __restrict__ fst, const R* __restrict__ dr_t, const R* __restrict__ u1,
          const R* __restrict__ phi1, const R* __restrict__ mu1, const R* __restrict__ lf1,
          const R* __restrict__ lu1, const R* __restrict__ lmu1, R* __restrict__ lf0,
          R* __restrict__ t_phil, R* __restrict__ w, R* __restrict__ lmu0, R tshift1, double* __restrict__ part) {
  double gpart[NG] = {0, 0, 0, 0, 0, 0};
  int64_t P;
  int x, y, z;
  if (adj_cell(p.n, p.sy, p.sz, P, x, y, z))
    adj_lbm_cell<D, Q, N, NC, R, TAPE>(p, P, x, y, z, fst, dr_t, u1, phi1, mu1, lf1, lu1, lmu1, lf0, t_phil, w,
                                       lmu0, tshift1, gpart);
  block_partials(gpart, part);
}

// ---------------------------------------------------------------------------
// 2-3. the mu update (gathered over the faces of each cell), then the
// projection and local phase-field terms of the same cell
// ---------------------------------------------------------------------------
template <int N, int NC, class R>
__device__ __forceinline__ void mu_quant(const KP<R>& p, const R (&ph)[N], const R (&m)[NC], R td,
                                         R (&M)[NC][NC], R (&cs)[NC]) {
  R h[N];
  interp_h<N, R>(ph, h);
#pragma unroll
  for (int i = 0; i < NC; ++i) {
    cs[i] = R(0);
#pragma unroll
    for (int k = 0; k < NC; ++k) M[i][k] = R(0);
  }
#pragma unroll
  for (int b = 0; b < N; ++b)
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      R C = p.c0s[b][i] + p.mT[b][i] * td;
#pragma unroll
      for (int k = 0; k < NC; ++k) C += p.chi[i][k] * m[k];
      cs[i] += h[b] * C;
#pragma unroll
      for (int k = 0; k < NC; ++k) M[i][k] += ph[b] * p.D[b][i] * p.chi[i][k];
    }
}

template <int D, int N, int NC, class R>
__device__ __forceinline__ void mu_adj_cell(const KP<R>& p, int64_t P, int x, int y, int z,
                                            const R* __restrict__ phi0, const R* __restrict__ phi1,
                                            const R* __restrict__ mu0, const R* __restrict__ mu1,
                                            const R* __restrict__ u0, const R* __restrict__ w, R tshift,
                                            R (&mub_o)[NC], R (&Ub_o)[D], R (&p1b_o)[N], R (&p0b_o)[N],
                                            double (&gpart)[NG]) {
  {
    const int pos[3] = {x, y, z};
    const int64_t stride[3] = {1, p.sy, p.sz};
    const int pa = p.pull_axis;
    const R tdP = tdev_at(p, pos[pa], tshift);
    R php[N], mp[NC], wp[NC], MP[NC][NC], cP[NC];
#pragma unroll
    for (int b = 0; b < N; ++b) php[b] = phi1[b * p.cells + P];
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      mp[i] = mu0[i * p.cells + P];
      wp[i] = w[i * p.cells + P];
    }
    mu_quant<N, NC, R>(p, php, mp, tdP, MP, cP);
    R mub[NC], Mb[NC][NC], cb[NC], Ub[D];
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      mub[i] = R(0);
      cb[i] = R(0);
#pragma unroll
      for (int k = 0; k < NC; ++k) Mb[i][k] = R(0);
    }
    const R conv = p.conv, idx = p.idx, dtdx = p.dt * p.idx;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      Ub[a] = R(0);
      const R uaP = u0[a * p.cells + P];
#pragma unroll
      for (int si = 0; si < 2; ++si) {
        const int s = si ? 1 : -1;
        // wall faces carry no flux: their seed is zeroed below rather than
        // branched around, so the loads of all faces can be issued together
        const bool wall = !p.per[a] && ((s < 0 && pos[a] == 0) || (s > 0 && pos[a] == p.n[a] - 1));
        const int q = nb_field(pos[a], s, p.n[a], p.per[a]);
        const int64_t Qj = P + (int64_t)(q - pos[a]) * stride[a];
        R phq[N], mq[NC], wq[NC], MQ[NC][NC], cQ[NC];
#pragma unroll
        for (int b = 0; b < N; ++b) phq[b] = phi1[b * p.cells + Qj];
#pragma unroll
        for (int i = 0; i < NC; ++i) {
          mq[i] = mu0[i * p.cells + Qj];
          wq[i] = w[i * p.cells + Qj];
        }
        mu_quant<N, NC, R>(p, phq, mq, a == pa ? tdev_at(p, q, tshift) : tdP, MQ, cQ);
        const R uaQ = u0[a * p.cells + Qj];
        // the face with left cell L and right cell R = L + e_a
        const R sgn = (s > 0) ? R(1) : R(-1);  // +1: this cell is L
        R Jb[NC], dmu[NC];
#pragma unroll
        for (int i = 0; i < NC; ++i) {
          Jb[i] = wall ? R(0) : dtdx * sgn * (wq[i] - wp[i]);
          dmu[i] = sgn * (mq[i] - mp[i]);  // mu_R - mu_L
        }
#pragma unroll
        for (int k = 0; k < NC; ++k)
#pragma unroll
          for (int i = 0; i < NC; ++i) {
            mub[k] += sgn * Jb[i] * R(0.5) * (MP[i][k] + MQ[i][k]) * idx;
            Mb[i][k] += Jb[i] * (-R(0.5) * dmu[k] * idx);
          }
#pragma unroll
        for (int i = 0; i < NC; ++i) {
          Ub[a] += Jb[i] * R(0.5) * conv * R(0.5) * (cP[i] + cQ[i]);
          cb[i] += Jb[i] * R(0.5) * (uaP + uaQ) * conv * R(0.5);
        }
      }
    }
    // source term and chi_tot at the cell
    R ph0[N], h0[N], h1[N];
#pragma unroll
    for (int b = 0; b < N; ++b) ph0[b] = phi0[b * p.cells + P];
    interp_h<N, R>(ph0, h0);
    interp_h<N, R>(php, h1);
    R chidm[NC];
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      chidm[i] = R(0);
#pragma unroll
      for (int k = 0; k < NC; ++k) chidm[i] += p.chi[i][k] * (mu1[k * p.cells + P] - mp[k]);
    }
    R wchidm = R(0);
#pragma unroll
    for (int i = 0; i < NC; ++i) wchidm += wp[i] * chidm[i];
    R h1b[N], h0b[N];
#pragma unroll
    for (int b = 0; b < N; ++b) {
      R wC = R(0), cC = R(0), wT = R(0);
#pragma unroll
      for (int i = 0; i < NC; ++i) {
        R C = p.c0s[b][i] + p.mT[b][i] * tdP;
#pragma unroll
        for (int k = 0; k < NC; ++k) C += p.chi[i][k] * mp[k];
        wC += wp[i] * C;
        cC += cb[i] * C;
        wT += wp[i] * p.mT[b][i];
      }
      // the dT/dt term -h1_b mT[b] (T^{n+1} - T^n) of the update
      h1b[b] = -wC - wchidm + cC - wT * p.dtdev;
      h0b[b] = wC;
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        R wchi = R(0), cchi = R(0);
#pragma unroll
        for (int i = 0; i < NC; ++i) {
          wchi += wp[i] * p.chi[i][j];
          cchi += cb[i] * p.chi[i][j];
        }
        mub[j] += -(h1[b] - h0[b]) * wchi + h1[b] * cchi;
      }
    }
    // M = sum_a phi_a diag(D_a) chi at phi^{n+1}
    R p1b[N];
#pragma unroll
    for (int b = 0; b < N; ++b) {
      R acc = R(0);
#pragma unroll
      for (int i = 0; i < NC; ++i)
#pragma unroll
        for (int k = 0; k < NC; ++k) acc += Mb[i][k] * p.D[b][i] * p.chi[i][k];
      p1b[b] = acc;
    }
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      R acc = R(0);
#pragma unroll
      for (int k = 0; k < NC; ++k) acc += Mb[i][k] * php[N - 1] * p.chi[i][k];
      gpart[G_D0 + i] = (double)acc;
    }
    // h chains
    R p0b[N];
#pragma unroll
    for (int g = 0; g < N; ++g) {
      R a1 = R(0), a0 = R(0);
#pragma unroll
      for (int b = 0; b < N; ++b) {
        a1 += h1b[b] * dh<N, R>(php, b, g);
        a0 += h0b[b] * dh<N, R>(ph0, b, g);
      }
      p1b[g] += a1;
      p0b[g] = a0;
    }
#pragma unroll
    for (int i = 0; i < NC; ++i) mub_o[i] = mub[i];
#pragma unroll
    for (int a = 0; a < D; ++a) Ub_o[a] = Ub[a];
#pragma unroll
    for (int b = 0; b < N; ++b) {
      p1b_o[b] = p1b[b];
      p0b_o[b] = p0b[b];
    }
  }
}

// ---------------------------------------------------------------------------
// 4. projection and the local phase-field terms
// ---------------------------------------------------------------------------
template <int D, int N, int NC, class R, bool ACT>
__global__ void __launch_bounds__(ADJ_BLOCK)
k_adj_muphi(KP<R> p, const R* __restrict__ phi0, const R* __restrict__ phi1,
            const R* __restrict__ mu0, const R* __restrict__ mu1, const R* __restrict__ u0,
            const R* __restrict__ w, const R* __restrict__ lphi1, const R* __restrict__ t_phil,
            R* __restrict__ lphi0, R* __restrict__ lmu0, R* __restrict__ lu0, R* __restrict__ rbar,
            uint8_t* __restrict__ rflag, uint8_t* __restrict__ rowflag, const uint8_t* __restrict__ act,
            R tshift, double* __restrict__ part) {
  double gpart[NG] = {0, 0, 0, 0, 0, 0};
  int64_t P;
  int x, y, z;
  if (adj_cell(p.n, p.sy, p.sz, P, x, y, z)) {
    R mubf[NC], Ubf[D], p1bf[N], p0bf[N];
    mu_adj_cell<D, N, NC, R>(p, P, x, y, z, phi0, phi1, mu0, mu1, u0, w, tshift, mubf, Ubf, p1bf, p0bf, gpart);
#pragma unroll
    for (int a = 0; a < D; ++a) lu0[a * p.cells + P] = Ubf[a];
    // the active set of phi^n: recorded by the forward recomputation of the
    // step (ACT), else from phi^n's 9/19-point stencil, which only the
    // interface cells need otherwise
    unsigned active = 0u;
    R v[N][3][3][3];
    if constexpr (ACT) {
      active = act[P];
    } else {
      load_stencil<D, N, R>(p, phi0, x, y, z, v);
      active = active_of<D, N, R>(v);
    }
    R pb[N];
#pragma unroll
    for (int b = 0; b < N; ++b) pb[b] = lphi1[b * p.cells + P] + p1bf[b];
    pb[N - 1] += t_phil[P];
    R p0b[N], Rb[N];
#pragma unroll
    for (int b = 0; b < N; ++b) {
      p0b[b] = p0bf[b];
      Rb[b] = R(0);
    }
    R mub[NC];
#pragma unroll
    for (int i = 0; i < NC; ++i) mub[i] = mubf[i];
    if (__builtin_popcount(active) <= 1) {
#pragma unroll
      for (int b = 0; b < N; ++b) p0b[b] += pb[b];
    } else {
      if constexpr (ACT) load_stencil<D, N, R>(p, phi0, x, y, z, v);
      R Rv[N], vv[N], out[N], theta;
      pf_rhs<D, N, NC, R>(p, v, mu0, x, y, z, tshift, Rv);
#pragma unroll
      for (int b = 0; b < N; ++b) vv[b] = v[b][1][1][1] + p.rate * Rv[b];
      project_masked<N, R>(active, vv, out, theta);
      unsigned supp = 0u;
      int ns = 0;
      R mean = R(0);
#pragma unroll
      for (int b = 0; b < N; ++b)
        if (((active >> b) & 1u) && vv[b] - theta > R(0)) {
          supp |= 1u << b;
          ++ns;
          mean += pb[b];
        }
      mean = mean / R(ns);
      R vb[N], taub = R(0);
      const R rtau = -p.rate / p.tau_pf;
#pragma unroll
      for (int b = 0; b < N; ++b) {
        vb[b] = ((supp >> b) & 1u) ? pb[b] - mean : R(0);
        p0b[b] += vb[b];
        Rb[b] = p.rate * vb[b];
        taub += vb[b] * Rv[b] * rtau;
      }
      gpart[G_TAU] += (double)taub;
      // local terms: -dW/dphi / eps and -sum psi dh/dphi
      R ph[N], m[NC];
#pragma unroll
      for (int b = 0; b < N; ++b) ph[b] = v[b][1][1][1];
#pragma unroll
      for (int i = 0; i < NC; ++i) m[i] = p.mu_ref[i] + mu0[i * p.cells + P];
#pragma unroll
      for (int al = 0; al < N; ++al)
#pragma unroll
        for (int be = 0; be < N; ++be) {
          if (be == al) continue;
          if (p.potential == 0) {
            p0b[be] += -Rb[al] * R(1.6211389382774044) * p.gamma[al][be] * p.ieps;  // 16 / pi^2
          } else {
            p0b[al] += -Rb[al] * R(18) * p.gamma[al][be] * ph[be] * ph[be] * p.ieps;
            p0b[be] += -Rb[al] * R(36) * p.gamma[al][be] * ph[al] * ph[be] * p.ieps;
          }
        }
      const R tdev = (p.G != R(0)) ? p.G * (R((p.pull_axis == 0) ? x : (p.pull_axis == 1 ? y : z)) - tshift)
                                   : p.tdev_iso;
      R ps[N], C[N][NC];
#pragma unroll
      for (int b = 0; b < N; ++b) {
        R r = R(0);
#pragma unroll
        for (int i = 0; i < NC; ++i) {
          R chimu = R(0);
#pragma unroll
          for (int j = 0; j < NC; ++j) chimu += p.chi[i][j] * m[j];
          r += -R(0.5) * m[i] * chimu - m[i] * (p.c0[b][i] + p.mT[b][i] * tdev);
          C[b][i] = p.c0[b][i] + p.mT[b][i] * tdev + chimu;
        }
        ps[b] = r + p.dS[b] * tdev;
      }
#pragma unroll
      for (int al = 0; al < N; ++al)
#pragma unroll
        for (int be = 0; be < N; ++be) {
          const R d1 = dh<N, R>(ph, be, al);
#pragma unroll
          for (int i = 0; i < NC; ++i) mub[i] += Rb[al] * d1 * C[be][i];
#pragma unroll
          for (int g = 0; g < N; ++g) p0b[g] += -Rb[al] * ps[be] * d2h<N, R>(ph, be, al, g);
        }
    }
#pragma unroll
    for (int i = 0; i < NC; ++i) lmu0[i * p.cells + P] += mub[i];
    bool nz = false;
#pragma unroll
    for (int b = 0; b < N; ++b) {
      lphi0[b * p.cells + P] = p0b[b];
      rbar[b * p.cells + P] = Rb[b];
      nz = nz || (Rb[b] != R(0));
    }
    rflag[P] = nz ? 1 : 0;
    // the (y, z) row holds a seed: every writer stores the same value
    if (nz) rowflag[(int64_t)z * p.n[1] + y] = 1;
  }
  block_partials(gpart, part);
}

// ---------------------------------------------------------------------------
// 5. face fluxes and cell-centre terms of the gradient energy
// ---------------------------------------------------------------------------

// position along one axis of a face owner or cell-term centre: periodic axes
// wrap, positions outside a wall do not exist
__device__ __forceinline__ bool owner_coord(int v, int n, int per, int& out) {
  if (v >= 0 && v < n) { out = v; return true; }
  if (!per) return false;
  out = ((v % n) + n) % n;
  return true;
}

// Reverse of one face flux J_a (left cell L, right cell L + e_a), seeded with
// Jb[phase]: the adjoints pfb of the face value of phi and grb of its face
// gradient, which give the contribution to the adjoint of phi at each role
// cell (0 L, 1 R, then per tangential axis b in order: L-e_b, L+e_b, R-e_b,
// R+e_b; face_store).  dd: derivative in delta (pairs with delta != 0).
template <int D, int N, class R>
__device__ __forceinline__ void face_vjp(const KP<R>& p, const R* __restrict__ phi, const int (&Lc)[3],
                                         int a, const R (&Jb)[N], R (&pfb)[N], R (&grb)[N][D], R& dd) {
  constexpr int NR = 2 + 4 * (D - 1);
  int rc[NR][3];
  int o[NR][3];
#pragma unroll
  for (int r = 0; r < NR; ++r) o[r][0] = o[r][1] = o[r][2] = 0;
  o[1][a] = 1;
  {
    int r = 2;
#pragma unroll
    for (int b = 0; b < D; ++b) {
      if (b == a) continue;
      o[r][b] = -1;
      o[r + 1][b] = 1;
      o[r + 2][a] = 1;
      o[r + 2][b] = -1;
      o[r + 3][a] = 1;
      o[r + 3][b] = 1;
      r += 4;
    }
  }
  R ph[NR][N];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
#pragma unroll
    for (int e = 0; e < 3; ++e)
      rc[r][e] = (e < D) ? nb_field(Lc[e], o[r][e], p.n[e], p.per[e]) : 0;
    const int64_t j = (int64_t)rc[r][2] * p.sz + (int64_t)rc[r][1] * p.sy + rc[r][0];
#pragma unroll
    for (int b = 0; b < N; ++b) ph[r][b] = phi[b * p.cells + j];
  }
  const R idx = R(1) / p.dx, ih2 = R(0.5) / p.dx;
  R pf[N], gr[N][D];
#pragma unroll
  for (int b = 0; b < N; ++b) {
    pf[b] = R(0.5) * (ph[0][b] + ph[1][b]);
    int r = 2;
#pragma unroll
    for (int e = 0; e < D; ++e) {
      if (e == a) {
        gr[b][e] = (ph[1][b] - ph[0][b]) * idx;
      } else {
        gr[b][e] = R(0.5) * ((ph[r + 1][b] - ph[r][b]) * ih2 + (ph[r + 3][b] - ph[r + 2][b]) * ih2);
        r += 4;
      }
    }
  }
#pragma unroll
  for (int b = 0; b < N; ++b) {
    pfb[b] = R(0);
#pragma unroll
    for (int e = 0; e < D; ++e) grb[b][e] = R(0);
  }
  dd = R(0);
#pragma unroll
  for (int al = 0; al < N; ++al)
#pragma unroll
    for (int be = al + 1; be < N; ++be) {
      if (Jb[al] == R(0) && Jb[be] == R(0)) continue;
      R q[D], g[D];
#pragma unroll
      for (int e = 0; e < D; ++e) q[e] = pf[al] * gr[be][e] - pf[be] * gr[al][e];
      dAdq<D, R, R>(q, p.gamma[al][be], p.delta[al][be], p.qmin2, g);
      pfb[be] += -Jb[al] * g[a];
      pfb[al] += Jb[be] * g[a];
      R gbv[D];
#pragma unroll
      for (int e = 0; e < D; ++e) gbv[e] = R(0);
      gbv[a] = -Jb[al] * pf[be] + Jb[be] * pf[al];
      R qb[D], ddl;
      dAdq_vjp<D, R>(q, p.gamma[al][be], p.delta[al][be], p.qmin2, gbv, qb, ddl);
      if (p.delta[al][be] != R(0)) dd += ddl;
#pragma unroll
      for (int e = 0; e < D; ++e) {
        pfb[al] += qb[e] * gr[be][e];
        pfb[be] -= qb[e] * gr[al][e];
        grb[be][e] += qb[e] * pf[al];
        grb[al][e] -= qb[e] * pf[be];
      }
    }
}

// The N (1 + D) values a face (a, L) stores for the gather, from its pfb, grb:
// k = b: the contribution to phi_b at role 0 (L), N + b: at role 1 (R),
// 2N + b (D - 1) + t: the one at the roles along the t-th tangential axis,
// with sign - at L-e, R-e and + at L+e, R+e.
template <int D, int N, class R>
__device__ __forceinline__ void face_store(const KP<R>& p, int a, const R (&pfb)[N], const R (&grb)[N][D],
                                           R* __restrict__ fb, int64_t L) {
  const R idx = R(1) / p.dx, ih2 = R(0.5) / p.dx;
#pragma unroll
  for (int b = 0; b < N; ++b) {
    fb[(int64_t)b * p.cells + L] = R(0.5) * pfb[b] - grb[b][a] * idx;
    fb[(int64_t)(N + b) * p.cells + L] = R(0.5) * pfb[b] + grb[b][a] * idx;
    int t = 0;
#pragma unroll
    for (int e = 0; e < D; ++e) {
      if (e == a) continue;
      fb[(int64_t)(2 * N + b * (D - 1) + t) * p.cells + L] = R(0.5) * grb[b][e] * ih2;
      ++t;
    }
  }
}
// Contribution of face (a, L) to the adjoint of phi_b at its role cell r
template <int D, int N, class R>
__device__ __forceinline__ R face_role(const KP<R>& p, const R* __restrict__ fb, int r, int b, int64_t L) {
  if (r < 2) return fb[(int64_t)(r * N + b) * p.cells + L];
  const int t = (r - 2) / 4, k = (r - 2) % 4;
  const R g = fb[(int64_t)(2 * N + b * (D - 1) + t) * p.cells + L];
  return (k % 2) ? g : -g;
}

// Reverse of the cell-centre term at P seeded with cb = -eps Rbar(P): the
// adjoints phb of phi at P and gcb of its central gradient, which give the
// contribution at each role cell (0 P, then per axis b: P-e_b, P+e_b;
// cell_store).
template <int D, int N, class R>
__device__ __forceinline__ void cell_vjp(const KP<R>& p, const R* __restrict__ phi, const int (&Pc)[3],
                                         const R (&cb)[N], R (&phb)[N], R (&gcb)[N][D], R& dd) {
  constexpr int NR = 1 + 2 * D;
  int rc[NR][3];
  R ph[NR][N];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      int off = 0;
      if (r > 0 && e == (r - 1) / 2) off = ((r - 1) % 2) ? 1 : -1;
      rc[r][e] = (e < D) ? nb_field(Pc[e], off, p.n[e], p.per[e]) : 0;
    }
    const int64_t j = (int64_t)rc[r][2] * p.sz + (int64_t)rc[r][1] * p.sy + rc[r][0];
#pragma unroll
    for (int b = 0; b < N; ++b) ph[r][b] = phi[b * p.cells + j];
  }
  const R ih2 = R(0.5) / p.dx;
  R gc[N][D];
#pragma unroll
  for (int b = 0; b < N; ++b) {
    phb[b] = R(0);
#pragma unroll
    for (int e = 0; e < D; ++e) {
      gc[b][e] = (ph[2 + 2 * e][b] - ph[1 + 2 * e][b]) * ih2;
      gcb[b][e] = R(0);
    }
  }
  dd = R(0);
#pragma unroll
  for (int al = 0; al < N; ++al)
#pragma unroll
    for (int be = al + 1; be < N; ++be) {
      if (cb[al] == R(0) && cb[be] == R(0)) continue;
      R q[D], g[D];
#pragma unroll
      for (int e = 0; e < D; ++e) q[e] = ph[0][al] * gc[be][e] - ph[0][be] * gc[al][e];
      dAdq<D, R, R>(q, p.gamma[al][be], p.delta[al][be], p.qmin2, g);
      R gbv[D];
#pragma unroll
      for (int e = 0; e < D; ++e) {
        gbv[e] = cb[al] * gc[be][e] - cb[be] * gc[al][e];
        gcb[be][e] += cb[al] * g[e];
        gcb[al][e] -= cb[be] * g[e];
      }
      R qb[D], ddl;
      dAdq_vjp<D, R>(q, p.gamma[al][be], p.delta[al][be], p.qmin2, gbv, qb, ddl);
      if (p.delta[al][be] != R(0)) dd += ddl;
#pragma unroll
      for (int e = 0; e < D; ++e) {
        phb[al] += qb[e] * gc[be][e];
        phb[be] -= qb[e] * gc[al][e];
        gcb[be][e] += qb[e] * ph[0][al];
        gcb[al][e] -= qb[e] * ph[0][be];
      }
    }
}

// The N (1 + D) values the cell term at P stores for the gather: k = b: the
// contribution to phi_b at role 0 (P), N + b D + e: the one at P+e_e (at
// P-e_e with sign -).
template <int D, int N, class R>
__device__ __forceinline__ void cell_store(const KP<R>& p, const R (&phb)[N], const R (&gcb)[N][D],
                                           R* __restrict__ cb, int64_t P) {
  const R ih2 = R(0.5) / p.dx;
#pragma unroll
  for (int b = 0; b < N; ++b) {
    cb[(int64_t)b * p.cells + P] = phb[b];
#pragma unroll
    for (int e = 0; e < D; ++e) cb[(int64_t)(N + b * D + e) * p.cells + P] = gcb[b][e] * ih2;
  }
}
// Contribution of the cell term at P to the adjoint of phi_b at its role cell r
template <int D, int N, class R>
__device__ __forceinline__ R cell_role(const KP<R>& p, const R* __restrict__ cb, int r, int b, int64_t P) {
  if (r == 0) return cb[(int64_t)b * p.cells + P];
  const int e = (r - 1) / 2;
  const R g = cb[(int64_t)(N + b * D + e) * p.cells + P];
  return ((r - 1) % 2) ? g : -g;
}

// 5a. Writer: every cell computes, once, the reverse of the face fluxes it
// owns (its +e_a faces) and of its cell-centre term, and stores the N (1 + D)
// values that give their contributions at the role cells: fbuf[a NFV + k][L],
// cbuf[k][P] (face_store, cell_store).  Only entries with a non-zero seed are
// written; fflag[a][L] / rflag[P] (written by k_adj_muphi) say which.
template <int D, int N, int NC, class R>
__global__ void __launch_bounds__(ADJ_BLOCK)
k_adj_vjp(KP<R> p, const R* __restrict__ phi0, const R* __restrict__ rbar,
          const uint8_t* __restrict__ rflag, R* __restrict__ fbuf, uint8_t* __restrict__ fflag,
          R* __restrict__ cbuf, double* __restrict__ part, const uint8_t* __restrict__ rowflag, int split) {
  constexpr int NFV = N * (1 + D);
  double gpart[NG] = {0, 0, 0, 0, 0, 0};
  // split: D + 1 linear grids side by side, grid a < D for the faces along a,
  // grid D for the cell terms (more waves in flight on small grids); else
  // every thread does all of its cell's items
  const unsigned nb = split ? gridDim.x / (unsigned)(D + 1) : gridDim.x;
  const int item = split ? (int)(blockIdx.x / nb) : -1;
  int64_t L;
  int lc[3];
  // the cell's faces and its cell term carry a seed only if its row or the
  // rows of its +y and +z neighbours hold one (row flags of k_adj_muphi)
  auto seeded_rows = [&](const int (&c3)[3]) {
    const int yn = nb_field(c3[1], 1, p.n[1], p.per[1]);
    bool r = rowflag[(int64_t)c3[2] * p.n[1] + c3[1]] | rowflag[(int64_t)c3[2] * p.n[1] + yn];
    if (D == 3) r = r | rowflag[(int64_t)nb_field(c3[2], 1, p.n[2], p.per[2]) * p.n[1] + c3[1]];
    return r;
  };
  const bool valid = adj_cell(p.n, p.sy, p.sz, L, lc[0], lc[1], lc[2], blockIdx.x % nb);
  if (valid && !seeded_rows(lc)) {
#pragma unroll
    for (int a = 0; a < D; ++a)
      if (item < 0 || item == a) fflag[(int64_t)a * p.cells + L] = 0;
  } else if (valid) {
    const int Lc[3] = {lc[0], lc[1], lc[2]};
    R rl[N];
#pragma unroll
    for (int b = 0; b < N; ++b) rl[b] = rbar[b * p.cells + L];
    R dd_sum = R(0);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      if (item >= 0 && item != a) continue;
      int rcoord = 0;
      bool has = owner_coord(Lc[a] + 1, p.n[a], p.per[a], rcoord);  // false: wall face
      uint8_t flag = 0;
      if (has) {
        int Rc[3] = {Lc[0], Lc[1], Lc[2]};
        Rc[a] = rcoord;
        const int64_t Rj = (int64_t)Rc[2] * p.sz + (int64_t)Rc[1] * p.sy + Rc[0];
        if (rflag[L] | rflag[Rj]) {
          R Jb[N];
          bool any = false;
#pragma unroll
          for (int b = 0; b < N; ++b) {
            Jb[b] = p.eps * (rl[b] - rbar[b * p.cells + Rj]) / p.dx;
            any = any || (Jb[b] != R(0));
          }
          if (any) {
            R pfb[N], grb[N][D], dd;
            face_vjp<D, N, R>(p, phi0, Lc, a, Jb, pfb, grb, dd);
            dd_sum += dd;
            face_store<D, N, R>(p, a, pfb, grb, fbuf + (int64_t)a * NFV * p.cells, L);
            flag = 1;
          }
        }
      }
      fflag[(int64_t)a * p.cells + L] = flag;
    }
    if ((item < 0 || item == D) && rflag[L]) {
      R cbv[N];
#pragma unroll
      for (int b = 0; b < N; ++b) cbv[b] = -p.eps * rl[b];
      R phb[N], gcb[N][D], dd;
      cell_vjp<D, N, R>(p, phi0, Lc, cbv, phb, gcb, dd);
      dd_sum += dd;
      cell_store<D, N, R>(p, phb, gcb, cbuf, L);
    }
    gpart[G_DELTA] = (double)dd_sum;
  }
  block_partials(gpart, part);
}

// role offsets (relative to the owner) of a face along a: 0 L, 1 R, then per
// tangential axis b: L-e_b, L+e_b, R-e_b, R+e_b
template <int D>
__device__ __forceinline__ int face_role_off(int a, int r, int e) {
  if (r == 0) return 0;
  if (r == 1) return e == a ? 1 : 0;
  const int t = (r - 2) / 4, k = (r - 2) % 4;  // t-th tangential axis
  int b = 0, cnt = -1;
  for (int q = 0; q < D; ++q)
    if (q != a && ++cnt == t) b = q;
  if (e == b) return (k % 2) ? 1 : -1;
  if (e == a) return (k >= 2) ? 1 : 0;
  return 0;
}

// 5b. Gather: lam phi^n(X) += every stored contribution whose role cell is X.
// Cells with no flagged seed in their 9/19-point neighbourhood return at once.
// rowflag: per (y, z) row, 1 if a cell of the row holds a seed (written by
// k_adj_muphi of this step); rowclear: the other step parity's row flags,
// cleared here (one thread per row) for the next reverse step.
template <int D, int N, int NC, class R>
__device__ __forceinline__ void adj_phi2_cell(const KP<R>& p, const int64_t X, const int (&xc)[3],
                                              const uint8_t* __restrict__ rflag, const R* __restrict__ fbuf,
                                              const uint8_t* __restrict__ fflag, const R* __restrict__ cbuf,
                                              R* __restrict__ lphi0, const uint8_t* __restrict__ rowflag,
                                              uint8_t* __restrict__ rowclear) {
  constexpr int NRF = 2 + 4 * (D - 1), NRC = 1 + 2 * D, NFV = N * (1 + D);
  if (xc[0] == 0) rowclear[(int64_t)xc[2] * p.n[1] + xc[1]] = 0;
  // no seed in the 3 x 3 rows (y, z) around the cell: nothing to gather
  bool row_any = false;
#pragma unroll
  for (int dz = (D == 3 ? -1 : 0); dz <= (D == 3 ? 1 : 0); ++dz)
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      const int yy = nb_field(xc[1], dy, p.n[1], p.per[1]);
      const int zz = (D == 3) ? nb_field(xc[2], dz, p.n[2], p.per[2]) : 0;
      row_any = row_any | (rowflag[(int64_t)zz * p.n[1] + yy] != 0);
    }
  if (!row_any) return;
  // every role offset, and every face's other cell, lies in the 9/19-point
  // neighbourhood (at most two non-zero components), so the 3D corners are skipped
  bool any = false;
#pragma unroll
  for (int dz = (D == 3 ? -1 : 0); dz <= (D == 3 ? 1 : 0); ++dz)
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        if (dx != 0 && dy != 0 && dz != 0) continue;
        const int xx = nb_field(xc[0], dx, p.n[0], p.per[0]);
        const int yy = nb_field(xc[1], dy, p.n[1], p.per[1]);
        const int zz = (D == 3) ? nb_field(xc[2], dz, p.n[2], p.per[2]) : 0;
        any = any | (rflag[(int64_t)zz * p.sz + (int64_t)yy * p.sy + xx] != 0);
      }
  if (!any) return;
  R acc[N];
#pragma unroll
  for (int b = 0; b < N; ++b) acc[b] = R(0);
  bool interior = true;
#pragma unroll
  for (int e = 0; e < D; ++e) interior = interior && xc[e] >= 1 && xc[e] <= p.n[e] - 2;
  if (interior) {
    // Away from walls and wraps every owner X - off(r) is a distinct cell and
    // its role r is the only one landing on X: the same sums in the same
    // order as the general path below, with every flag load issued at once.
    uint8_t ff[D][NRF], cf[NRC];
    int64_t Lj[D][NRF], Pj[NRC];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int r = 0; r < NRF; ++r) {
        int64_t o = face_role_off<D>(a, r, 0) + (int64_t)face_role_off<D>(a, r, 1) * p.sy;
        if (D == 3) o += (int64_t)face_role_off<D>(a, r, 2) * p.sz;
        Lj[a][r] = X - o;
        ff[a][r] = fflag[(int64_t)a * p.cells + Lj[a][r]];
      }
#pragma unroll
    for (int r = 0; r < NRC; ++r) {
      int64_t o = 0;
      if (r > 0) {
        const int e = (r - 1) / 2;
        o = (((r - 1) % 2) ? 1 : -1) * (e == 0 ? (int64_t)1 : (e == 1 ? p.sy : p.sz));
      }
      Pj[r] = X - o;
      cf[r] = rflag[Pj[r]];
    }
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int r = 0; r < NRF; ++r)
        if (ff[a][r])
#pragma unroll
          for (int b = 0; b < N; ++b)
            acc[b] += face_role<D, N, R>(p, fbuf + (int64_t)a * NFV * p.cells, r, b, Lj[a][r]);
#pragma unroll
    for (int r = 0; r < NRC; ++r)
      if (cf[r])
#pragma unroll
        for (int b = 0; b < N; ++b) acc[b] += cell_role<D, N, R>(p, cbuf, r, b, Pj[r]);
#pragma unroll
    for (int b = 0; b < N; ++b) lphi0[b * p.cells + X] += acc[b];
    return;
  }
  // faces: owners L = X - (role offset), deduplicated (periodic axes of 1 or 2 cells alias)
  for (int a = 0; a < D; ++a) {
    int64_t seen[NRF];
    int nseen = 0;
    for (int r0 = 0; r0 < NRF; ++r0) {
      int Lc[3] = {0, 0, 0};
      bool ok = true;
      for (int e = 0; e < D; ++e) ok = ok && owner_coord(xc[e] - face_role_off<D>(a, r0, e), p.n[e], p.per[e], Lc[e]);
      if (!ok) continue;
      const int64_t Lj = (int64_t)Lc[2] * p.sz + (int64_t)Lc[1] * p.sy + Lc[0];
      bool dup = false;
      for (int i = 0; i < nseen; ++i) dup = dup || (seen[i] == Lj);
      if (dup) continue;
      seen[nseen++] = Lj;
      if (!fflag[(int64_t)a * p.cells + Lj]) continue;
      for (int r = 0; r < NRF; ++r) {
        bool hit = true;
        for (int e = 0; e < D; ++e)
          hit = hit && (nb_field(Lc[e], face_role_off<D>(a, r, e), p.n[e], p.per[e]) == xc[e]);
        if (hit)
          for (int b = 0; b < N; ++b) acc[b] += face_role<D, N, R>(p, fbuf + (int64_t)a * NFV * p.cells, r, b, Lj);
      }
    }
  }
  // cell-centre terms: centres P = X - (role offset)
  {
    int64_t seen[NRC];
    int nseen = 0;
    for (int r0 = 0; r0 < NRC; ++r0) {
      int Pc[3] = {0, 0, 0};
      bool ok = true;
      for (int e = 0; e < D; ++e) {
        const int off = (r0 > 0 && e == (r0 - 1) / 2) ? (((r0 - 1) % 2) ? 1 : -1) : 0;
        ok = ok && owner_coord(xc[e] - off, p.n[e], p.per[e], Pc[e]);
      }
      if (!ok) continue;
      const int64_t Pj = (int64_t)Pc[2] * p.sz + (int64_t)Pc[1] * p.sy + Pc[0];
      bool dup = false;
      for (int i = 0; i < nseen; ++i) dup = dup || (seen[i] == Pj);
      if (dup) continue;
      seen[nseen++] = Pj;
      if (!rflag[Pj]) continue;
      for (int r = 0; r < NRC; ++r) {
        bool hit = true;
        for (int e = 0; e < D; ++e) {
          const int off = (r > 0 && e == (r - 1) / 2) ? (((r - 1) % 2) ? 1 : -1) : 0;
          hit = hit && (nb_field(Pc[e], off, p.n[e], p.per[e]) == xc[e]);
        }
        if (hit)
          for (int b = 0; b < N; ++b) acc[b] += cell_role<D, N, R>(p, cbuf, r, b, Pj);
      }
    }
  }
#pragma unroll
  for (int b = 0; b < N; ++b) lphi0[b * p.cells + X] += acc[b];
}

template <int D, int N, int NC, class R>
__global__ void __launch_bounds__(ADJ_BLOCK)
k_adj_phi2(KP<R> p, const uint8_t* __restrict__ rflag, const R* __restrict__ fbuf,
           const uint8_t* __restrict__ fflag, const R* __restrict__ cbuf, R* __restrict__ lphi0,
           const uint8_t* __restrict__ rowflag, uint8_t* __restrict__ rowclear) {
  int64_t X;
  int xc[3];
  if (adj_cell(p.n, p.sy, p.sz, X, xc[0], xc[1], xc[2]))
    adj_phi2_cell<D, N, NC, R>(p, X, xc, rflag, fbuf, fflag, cbuf, lphi0, rowflag, rowclear);
}

// 5b + 1 of the step before.  The streaming/collision reverse of step n - 1
// reads the adjoint populations, mu and U of step n, which k_adj_lbm and
// k_adj_muphi of step n wrote, but not lam phi^n: so it runs in the same
// launch as the gather of step n (one kernel boundary less per step).  The
// launch is two linear grids side by side: the first gathers, the second runs
// the LBM reverse, so neither waits for the other.
template <int D, int Q, int N, int NC, class R, bool TAPE>
__global__ void __launch_bounds__(ADJ_BLOCK)
k_adj_phi2_lbm(KP<R> p, const uint8_t* __restrict__ rflag, const R* __restrict__ fbuf,
               const uint8_t* __restrict__ fflag, const R* __restrict__ cbuf, R* __restrict__ lphi0,
               const uint8_t* __restrict__ rowflag, uint8_t* __restrict__ rowclear, const R* __restrict__ fst, const R* __restrict__ dr_t, const R* __restrict__ u1,
               const R* __restrict__ phi1, const R* __restrict__ mu1, const R* __restrict__ lf1,
               const R* __restrict__ lu1, const R* __restrict__ lmu1, R* __restrict__ lf0,
               R* __restrict__ t_phil, R* __restrict__ w, R* __restrict__ lmu0, R tshift1,
               double* __restrict__ part) {
  const unsigned nb = gridDim.x / 2u;
  int64_t P;
  int xc[3];
  if (blockIdx.x < nb) {
    if (adj_cell(p.n, p.sy, p.sz, P, xc[0], xc[1], xc[2], blockIdx.x))
      adj_phi2_cell<D, N, NC, R>(p, P, xc, rflag, fbuf, fflag, cbuf, lphi0, rowflag, rowclear);
  } else {
    const unsigned blk = blockIdx.x - nb;
    double gpart[NG] = {0, 0, 0, 0, 0, 0};
    if (adj_cell(p.n, p.sy, p.sz, P, xc[0], xc[1], xc[2], blk))
      adj_lbm_cell<D, Q, N, NC, R, TAPE>(p, P, xc[0], xc[1], xc[2], fst, dr_t, u1, phi1, mu1, lf1, lu1, lmu1,
                                         lf0, t_phil, w, lmu0, tshift1, gpart);
    block_partials(gpart, part, blk);
  }
}

// Sum the per-block running sums of the reverse sweep in a fixed order: each
// of GA blocks sums a contiguous slice, then one block adds the GA slice sums
// to the FP64 accumulators.
constexpr int GA = 256;
__global__ void __launch_bounds__(ADJ_BLOCK)
k_grad_slices(const double* __restrict__ part, int64_t nrows, double* __restrict__ slices) {
  __shared__ double sh[ADJ_BLOCK];
  const int64_t per = (nrows + GA - 1) / GA;
  const int64_t r0 = (int64_t)blockIdx.x * per, r1 = min(nrows, r0 + per);
  for (int i = 0; i < NG; ++i) {
    double s = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += ADJ_BLOCK) s += part[r * NG + i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int st = ADJ_BLOCK / 2; st > 0; st >>= 1) {
      if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) slices[blockIdx.x * NG + i] = sh[0];
    __syncthreads();
  }
}
__global__ void __launch_bounds__(GA)
k_grad_accum(const double* __restrict__ slices, double* __restrict__ acc) {
  __shared__ double sh[GA];
  for (int i = 0; i < NG; ++i) {
    sh[threadIdx.x] = slices[threadIdx.x * NG + i];
    __syncthreads();
    for (int st = GA / 2; st > 0; st >>= 1) {
      if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) acc[i] += sh[0];
    __syncthreads();
  }
}

template <class R>
__global__ void k_fill(R* __restrict__ a, int64_t n, R v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

}  // namespace gpf
