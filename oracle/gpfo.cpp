/*
 * gpfo.cpp -- FP64 CPU oracle of the coupled Grand-Potential phase-field /
 * lattice-Boltzmann time step.
 *
 * TEST INFRASTRUCTURE ONLY (see gpfo.h).  Plain loops over cells, one
 * sub-step after the other, in the order of Algorithm phfLBM (App. A):
 *   S0 temperature, S1 active set, S2 phase-field right-hand side,
 *   S3 simplex projection  (Eq. PhfGrand, Eq. Wpot, Sec. 2.1)
 *   S4 chemical potential  (Eq. conc)
 *   S5 forces, moments, BGK collision (Eqs. LBMEq_1, f^eq, discreteForce,
 *      drag G_D, buoyancy, rhovel)
 *   S6 streaming with half-way bounce-back.
 * No blocking, fusion or reordering.  The scalar type S is double, or
 * std::complex<double> for complex-step derivatives; every branch decides on
 * the real part.
 *
 * Parity pins: every function here is pinned by a test under tests/ against
 * a closed form, an identity, brute force or a published property; the
 * coupled dendrite/eutectic morphology, the value of the drag constant h and
 * the intended sign of buoyancy are parity unpinned (they rest on the
 * readings listed in the design doc).
 */
#include "gpfo.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

typedef std::complex<double> cplx;

inline double re(double x) { return x; }
inline double re(const cplx& z) { return z.real(); }

const double PI = 3.14159265358979323846;
constexpr int NP = 4; /* most phases (three solids and the liquid) */

/* ---------------- lattices (Table LBM_Schemes; D3Q19 textbook) ------------- */

struct Lattice {
  int Q;
  int c[27][3];
  double w[27];
  int opp[27];
};

/* Q = 9 (2D), 19 or 27 (3D) */
Lattice make_lattice_q(int Q) {
  Lattice L;
  std::memset(&L, 0, sizeof(L));
  if (Q == 27) {
    /* D3Q27 of Table LBM_Schemes: rest 8/27, 6 faces 2/27, 12 edges 1/54,
     * 8 corners 1/216.  Numbering: the D3Q19 directions first (same order),
     * then the corners in opposite pairs. */
    L.Q = 27;
    int k = 0;
    const int order19[19][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},
                                {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                                {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                                {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
    const int corners[8][3] = {{1, 1, 1},  {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1},
                               {1, -1, 1}, {-1, 1, -1},  {-1, 1, 1}, {1, -1, -1}};
    for (; k < 19; ++k)
      for (int a = 0; a < 3; ++a) L.c[k][a] = order19[k][a];
    for (int j = 0; j < 8; ++j, ++k)
      for (int a = 0; a < 3; ++a) L.c[k][a] = corners[j][a];
    for (k = 0; k < 27; ++k) {
      int len2 = L.c[k][0] * L.c[k][0] + L.c[k][1] * L.c[k][1] + L.c[k][2] * L.c[k][2];
      L.w[k] = len2 == 0 ? 8.0 / 27.0 : (len2 == 1 ? 2.0 / 27.0 : (len2 == 2 ? 1.0 / 54.0 : 1.0 / 216.0));
    }
  } else if (Q == 9) {
    /* numbering of the paper's D2Q9 figure; weights 4/9, 1/9, 1/36 */
    const int c2[9][2] = {{0, 0}, {1, 0}, {0, 1}, {-1, 0}, {0, -1},
                          {1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
    L.Q = 9;
    for (int k = 0; k < 9; ++k) {
      L.c[k][0] = c2[k][0];
      L.c[k][1] = c2[k][1];
      L.c[k][2] = 0;
      L.w[k] = (k == 0) ? 4.0 / 9.0 : (k <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
    }
  } else {
    /* D3Q19: rest, 6 faces (1/18), 12 edges (1/36); rest weight 1/3 */
    const int c3[19][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},
                           {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                           {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                           {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
    L.Q = 19;
    for (int k = 0; k < 19; ++k) {
      for (int a = 0; a < 3; ++a) L.c[k][a] = c3[k][a];
      int len2 = c3[k][0] * c3[k][0] + c3[k][1] * c3[k][1] + c3[k][2] * c3[k][2];
      L.w[k] = (len2 == 0) ? 1.0 / 3.0 : (len2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
  }
  /* opposite direction: the k with c_k = -c_j, found by search */
  for (int j = 0; j < L.Q; ++j)
    for (int k = 0; k < L.Q; ++k)
      if (L.c[k][0] == -L.c[j][0] && L.c[k][1] == -L.c[j][1] && L.c[k][2] == -L.c[j][2])
        L.opp[j] = k;
  return L;
}

Lattice make_lattice(int dim) { return make_lattice_q(dim == 2 ? 9 : 19); }

/* ---------------- parameters with the scalar type S ------------------------ */

template <class S>
struct Par {
  int dim, N, nc, potential, periodic[3], pull_axis, grav_axis, grav_sign;
  long n[3];
  S dx, dt, eps, tau_pf, gamma[NP][NP], delta[NP][NP], chi[2][2], c0[NP][2], dS[NP], T_E, T_iso,
      D[NP][2], G, V, y0, tau_lb, rho0, gbeta[2], c_ref[2], h_drag, W0, lid_u, eta[NP], mT[NP][2];
  long frame_every, frame_front;
};

template <class S>
Par<S> lift(const gpfo_params& p) {
  Par<S> q;
  q.dim = p.dim;
  q.N = p.N;
  q.nc = p.nc;
  q.potential = p.potential;
  q.pull_axis = p.pull_axis;
  q.grav_axis = p.grav_axis;
  q.grav_sign = p.grav_sign;
  for (int a = 0; a < 3; ++a) {
    q.periodic[a] = p.periodic[a];
    q.n[a] = (a < p.dim) ? (long)p.n[a] : 1;
  }
  q.dx = p.dx;
  q.dt = p.dt;
  q.eps = p.eps;
  q.tau_pf = p.tau_pf;
  for (int a = 0; a < NP; ++a)
    for (int b = 0; b < NP; ++b) {
      q.gamma[a][b] = p.gamma[a][b];
      q.delta[a][b] = p.delta[a][b];
    }
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) q.chi[i][j] = p.chi[i][j];
  for (int a = 0; a < NP; ++a) {
    for (int i = 0; i < 2; ++i) {
      q.c0[a][i] = p.c0[a][i];
      q.D[a][i] = p.D[a][i];
    }
    q.dS[a] = p.dS[a];
  }
  q.T_E = p.T_E;
  q.T_iso = p.T_iso;
  q.G = p.G;
  q.V = p.V;
  q.y0 = p.y0;
  q.tau_lb = p.tau_lb;
  q.rho0 = p.rho0;
  for (int i = 0; i < 2; ++i) {
    q.gbeta[i] = p.gbeta[i];
    q.c_ref[i] = p.c_ref[i];
  }
  q.h_drag = p.h_drag;
  q.W0 = p.W0;
  q.lid_u = p.lid_u;
  for (int a = 0; a < NP; ++a) q.eta[a] = p.eta[a];
  for (int a = 0; a < NP; ++a)
    for (int i = 0; i < 2; ++i) q.mT[a][i] = p.mT[a][i];
  q.frame_every = (long)p.frame_every;
  q.frame_front = (long)p.frame_front;
  return q;
}

/* ---------------- pointwise model functions -------------------------------- */

/* Cubic anisotropy function of a pair normal q (reading of the gradient
 * energy a(phi, grad phi), which the paper does not write out):
 *   a_c(q) = 1 - delta (3 - 4 sum_a q_a^4 / |q|^4),
 * which in 2D equals 1 + delta cos(4 theta).  Below |q|^2 = 1e-24 the
 * direction is undefined and a_c = 1. */
template <class S>
S aniso_ac(int dim, const S* q, S delta) {
  S q2 = 0, q4 = 0;
  for (int a = 0; a < dim; ++a) {
    q2 += q[a] * q[a];
    q4 += q[a] * q[a] * q[a] * q[a];
  }
  if (re(q2) <= 1e-24) return S(1.0);
  return S(1.0) - delta * (S(3.0) - S(4.0) * q4 / (q2 * q2));
}

/* Pair gradient energy A(q) = gamma a_c(q)^2 |q|^2. */
template <class S>
S aniso_A(int dim, const S* q, S gamma, S delta) {
  S q2 = 0;
  for (int a = 0; a < dim; ++a) q2 += q[a] * q[a];
  S ac = aniso_ac(dim, q, delta);
  return gamma * ac * ac * q2;
}

/* dA/dq = 2 gamma a_c (a_c q + |q|^2 grad_q a_c),
 * grad_q a_c = 16 delta (q_a^3 / |q|^4 - q_a sum_b q_b^4 / |q|^6). */
template <class S>
void aniso_dAdq(int dim, const S* q, S gamma, S delta, S* out) {
  S q2 = 0, q4 = 0;
  for (int a = 0; a < dim; ++a) {
    q2 += q[a] * q[a];
    q4 += q[a] * q[a] * q[a] * q[a];
  }
  if (re(q2) <= 1e-24) {
    for (int a = 0; a < dim; ++a) out[a] = S(2.0) * gamma * q[a];
    return;
  }
  S ac = S(1.0) - delta * (S(3.0) - S(4.0) * q4 / (q2 * q2));
  for (int a = 0; a < dim; ++a) {
    S grad_ac = S(16.0) * delta *
                (q[a] * q[a] * q[a] / (q2 * q2) - q[a] * q4 / (q2 * q2 * q2));
    out[a] = S(2.0) * gamma * ac * (ac * q[a] + q2 * grad_ac);
  }
}

/* Interpolation functions h_a(phi) (the paper uses h without defining it):
 * N = 2: h_a = phi_a^2 (3 - 2 phi_a);
 * N = 3: h_a = phi_a^2 (3 - 2 phi_a) + 2 phi_a phi_b phi_g;
 * N = 4: h_a = phi_a^2 (3 - 2 phi_a) + 2 phi_a sum_{b < g, both != a} phi_b phi_g.
 * All sum to 1 on the Gibbs simplex (3 p2 - 2 p3 + 6 e3 = 1 when e1 = 1).
 * dh[b*N + a] = d h_b / d phi_a. */
template <class S>
void interp_h(int N, const S* phi, S* h, S* dh) {
  for (int b = 0; b < N; ++b) {
    h[b] = phi[b] * phi[b] * (S(3.0) - S(2.0) * phi[b]);
    for (int a = 0; a < N; ++a) dh[b * N + a] = S(0.0);
    dh[b * N + b] = S(6.0) * phi[b] * (S(1.0) - phi[b]);
  }
  if (N >= 3) {
    /* + 2 phi_b e_b, e_b = sum over the pairs {g < k} of the other phases of
     * phi_g phi_k (for N = 3 the single product of the other two) */
    for (int b = 0; b < N; ++b) {
      S e = S(0.0);
      for (int g = 0; g < N; ++g)
        for (int k = g + 1; k < N; ++k)
          if (g != b && k != b) e += phi[g] * phi[k];
      h[b] += S(2.0) * phi[b] * e;
      dh[b * N + b] += S(2.0) * e;
      for (int a = 0; a < N; ++a) {
        if (a == b) continue;
        /* d e_b / d phi_a = sum of the phases other than a and b */
        S rest = S(0.0);
        for (int g = 0; g < N; ++g)
          if (g != a && g != b) rest += phi[g];
        dh[b * N + a] += S(2.0) * phi[b] * rest;
      }
    }
  }
}

/* Euclidean projection of v (m entries) onto the simplex {sum = 1, >= 0}:
 * the Lagrange multiplier of the constraint sum phi = 1 together with the
 * obstacle W = infinity off the Gibbs simplex (Sec. 2.1).  Sort-based
 * algorithm of Held, Wolfe and Crowder (1974): sort descending, take the
 * largest j with u_j - (sum_{i<=j} u_i - 1)/j > 0, theta = (sum - 1)/j. */
template <class S>
void project_simplex(int m, const S* v, S* out) {
  std::vector<S> u(v, v + m);
  std::sort(u.begin(), u.end(), [](const S& x, const S& y) { return re(x) > re(y); });
  S csum = 0, theta = 0;
  for (int j = 1; j <= m; ++j) {
    csum += u[j - 1];
    S t = (csum - S(1.0)) / S((double)j);
    if (re(u[j - 1] - t) > 0.0) theta = t;
  }
  for (int i = 0; i < m; ++i) out[i] = (re(v[i] - theta) > 0.0) ? v[i] - theta : S(0.0);
}

/* grand potential density of phase a (parabolic reading of the thermodynamics):
 * psi^a(mu, T) = -1/2 mu.chi.mu - mu.c0_a(T) + dS[a] (T - T_E), with the
 * parabola centre c0_a(T) = c0[a] + mT[a] (T - T_E): the equilibrium
 * composition of phase a moving along its coexistence line of App. B, whose
 * slopes are read as dc/dT (a slope 0 then means a composition independent
 * of T; read as dT/dc, a 0 would be an infinite rate).  It satisfies
 * -d psi^a / d mu = C^a(mu, T) = c0_a(T) + chi mu. */
template <class S>
S psi(const Par<S>& p, int a, const S* mu, S T) {
  S r = S(0.0);
  for (int i = 0; i < p.nc; ++i) {
    S chimu = 0;
    for (int j = 0; j < p.nc; ++j) chimu += p.chi[i][j] * mu[j];
    r += -S(0.5) * mu[i] * chimu - mu[i] * (p.c0[a][i] + p.mT[a][i] * (T - p.T_E));
  }
  return r + p.dS[a] * (T - p.T_E);
}

/* composition of phase a at (mu, T): C^a = c0[a] + mT[a] (T - T_E) + chi mu */
template <class S>
void comp_C(const Par<S>& p, int a, const S* mu, S T, S* C) {
  for (int i = 0; i < p.nc; ++i) {
    C[i] = p.c0[a][i] + p.mT[a][i] * (T - p.T_E);
    for (int j = 0; j < p.nc; ++j) C[i] += p.chi[i][j] * mu[j];
  }
}

/* f^eq of Eq. (f^eq) with c_s^2 = 1/3 (the printed factors are garbled):
 * w rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u). */
template <class S>
S feq(const Lattice& L, int k, S rho, const S* u, int dim) {
  S cu = 0, uu = 0;
  for (int a = 0; a < dim; ++a) {
    cu += S((double)L.c[k][a]) * u[a];
    uu += u[a] * u[a];
  }
  return L.w[k] * rho * (S(1.0) + S(3.0) * cu + S(4.5) * cu * cu - S(1.5) * uu);
}

/* Discrete force of Eq. (discreteForce) read as Guo's scheme:
 * (1 - 1/(2 tau)) w [3 (c - u) + 9 (c.u) c] . F. */
template <class S>
S guo(const Lattice& L, int k, S tau, const S* u, const S* F, int dim) {
  S cu = 0;
  for (int a = 0; a < dim; ++a) cu += S((double)L.c[k][a]) * u[a];
  S r = 0;
  for (int a = 0; a < dim; ++a) {
    S ca = S((double)L.c[k][a]);
    r += (S(3.0) * (ca - u[a]) + S(9.0) * cu * ca) * F[a];
  }
  return (S(1.0) - S(0.5) / tau) * L.w[k] * r;
}

/* ---------------- grid helpers --------------------------------------------- */

struct Grid {
  int dim;
  long n[3];
  int periodic[3];
  long cells() const { return n[0] * n[1] * n[2]; }
  long idx(long x, long y, long z) const { return (z * n[1] + y) * n[0] + x; }
  void coords(long i, long* x) const {
    x[0] = i % n[0];
    x[1] = (i / n[0]) % n[1];
    x[2] = i / (n[0] * n[1]);
  }
  /* neighbour index for field values: periodic axes wrap, walls mirror the
   * adjacent cell (zero normal derivative, the Neumann conditions of Case 1) */
  long field_nb(const long* x, const int* off) const {
    long y[3];
    for (int a = 0; a < 3; ++a) {
      y[a] = x[a] + off[a];
      if (y[a] < 0) y[a] = periodic[a] ? y[a] + n[a] : 0;
      if (y[a] >= n[a]) y[a] = periodic[a] ? y[a] - n[a] : n[a] - 1;
    }
    return idx(y[0], y[1], y[2]);
  }
  /* true when x + off stays inside the domain after periodic wrapping */
  bool inside(const long* x, const int* off, long* out) const {
    for (int a = 0; a < 3; ++a) {
      long y = x[a] + off[a];
      if (y < 0 || y >= n[a]) {
        if (!periodic[a]) return false;
        y = (y + n[a]) % n[a];
      }
      out[a] = y;
    }
    return true;
  }
};

/* ---------------- state ----------------------------------------------------- */

template <class S>
struct State {
  std::vector<S> phi, mu, f, u; /* [N][cells], [nc][cells], [Q][cells], [dim][cells] */
  long step;
  long shift = 0;               /* moving frame: cells shifted so far along the pull axis */
};

}  // namespace

struct gpfo_sim {
  gpfo_params prm;
  Grid g;
  Lattice L;
  State<double> st;
};

namespace {

/* ---------------- S0: temperature ------------------------------------------ */
/* Frozen temperature pulled at V cells per step (Case 2/3 setting):
 * T = T_E + G (x_pull + shift - y0 - V n), x_pull + shift the laboratory
 * coordinate when a moving frame has shifted the fields by `shift` cells;
 * isothermal runs (G = 0) use T_iso. */
template <class S>
S temperature(const Par<S>& p, const long* x, long nstep, long shift) {
  if (re(p.G) == 0.0) return p.T_iso;
  return p.T_E + p.G * (S((double)(x[p.pull_axis] + shift)) - p.y0 - p.V * S((double)nstep));
}

/* ---------------- S1: active set -------------------------------------------- */
/* A(P): phases that are non-zero somewhere in the lattice neighbourhood of P
 * (9 points in 2D, 19 in 3D).  Reading of the multiplier Lambda: the simplex
 * projection acts only on these phases, so no phase can appear in a cell
 * none of its neighbours holds.  With the D3Q27 lattice the phase-field
 * neighbourhood stays the 19 points (the corners carry no phase-field
 * coupling): the lattice only changes the populations. */
template <class S>
unsigned active_set(const Grid& g, const Lattice& L, const Par<S>& p, const State<S>& st,
                    const long* x) {
  unsigned mask = 0;
  long nc = g.cells();
  for (int k = 0; k < L.Q; ++k) {
    if (L.c[k][0] != 0 && L.c[k][1] != 0 && L.c[k][2] != 0) continue;
    long j = g.field_nb(x, L.c[k]);
    for (int a = 0; a < p.N; ++a)
      if (re(st.phi[a * nc + j]) > 0.0) mask |= 1u << a;
  }
  return mask;
}

/* ---------------- S2 + S3: phase field --------------------------------------- */

template <class S>
S phi_at(const Grid& g, const State<S>& st, int a, const long* x, int ox, int oy, int oz) {
  int off[3] = {ox, oy, oz};
  return st.phi[a * g.cells() + g.field_nb(x, off)];
}

/* central difference (phi(X + e_b) - phi(X - e_b)) / (2 dx) at X = x + o */
template <class S>
S grad_c(const Grid& g, const Par<S>& p, const State<S>& st, int a, const long* x, const int* o,
         int b) {
  int op[3] = {o[0], o[1], o[2]}, om[3] = {o[0], o[1], o[2]};
  op[b] += 1;
  om[b] -= 1;
  return (phi_at(g, st, a, x, op[0], op[1], op[2]) - phi_at(g, st, a, x, om[0], om[1], om[2])) /
         (S(2.0) * p.dx);
}

/* Right-hand side R_a of Eq. (PhfGrand) divided by nothing (tau eps dphi/dt = R):
 *   R_a = eps [ div J_a - sum_b dA_ab/dq(q_ab(P)) . grad phi_b(P) ]
 *         - (1/eps) dW/dphi_a - sum_b psi^b dh_b/dphi_a,
 * with the gradient energy a = sum_{a<b} A_ab(q_ab), q_ab = phi_a grad phi_b - phi_b grad phi_a,
 * J_a = d a / d grad phi_a = -sum_b phi_b dA_ab/dq evaluated on cell faces.
 * Face between P and Q = P + s e_a: phi_f = (phi_P + phi_Q)/2, normal
 * derivative s (phi_Q - phi_P)/dx, tangential derivatives the mean of the
 * central differences at P and Q.  Faces on walls carry no flux. */
template <class S>
void pf_rhs(const Grid& g, const Par<S>& p, const State<S>& st, const long* x, long nstep,
            S* R) {
  const int d = p.dim, N = p.N;
  const long nc_ = g.cells();
  const long P = g.idx(x[0], x[1], x[2]);
  S div[NP] = {};
  for (int a = 0; a < d; ++a) {
    for (int s = -1; s <= 1; s += 2) {
      long xq = x[a] + s;
      if (!p.periodic[a] && (xq < 0 || xq >= g.n[a])) continue; /* wall face: J = 0 */
      int oq[3] = {0, 0, 0};
      oq[a] = s;
      int o0[3] = {0, 0, 0};
      S phif[NP], grf[NP][3];
      for (int b = 0; b < N; ++b) {
        S pP = st.phi[b * nc_ + P];
        S pQ = phi_at(g, st, b, x, oq[0], oq[1], oq[2]);
        phif[b] = S(0.5) * (pP + pQ);
        for (int e = 0; e < d; ++e) {
          if (e == a)
            grf[b][e] = S((double)s) * (pQ - pP) / p.dx;
          else
            grf[b][e] = S(0.5) * (grad_c(g, p, st, b, x, o0, e) + grad_c(g, p, st, b, x, oq, e));
        }
      }
      for (int al = 0; al < N; ++al) {
        S J = 0; /* component a of J_al on this face */
        for (int be = 0; be < N; ++be) {
          if (be == al) continue;
          S q[3], dA[3];
          for (int e = 0; e < d; ++e) q[e] = phif[al] * grf[be][e] - phif[be] * grf[al][e];
          aniso_dAdq(d, q, p.gamma[al][be], p.delta[al][be], dA);
          J += -phif[be] * dA[a];
        }
        /* outward face (s = +1) adds, inward face subtracts */
        div[al] += S((double)s) * J / p.dx;
      }
    }
  }
  /* cell-centre term d a / d phi_a = sum_b dA_ab/dq . grad phi_b */
  S gc[NP][3];
  int o0[3] = {0, 0, 0};
  S phiP[NP];
  for (int b = 0; b < N; ++b) {
    phiP[b] = st.phi[b * nc_ + P];
    for (int e = 0; e < d; ++e) gc[b][e] = grad_c(g, p, st, b, x, o0, e);
  }
  S mu[2];
  for (int i = 0; i < p.nc; ++i) mu[i] = st.mu[i * nc_ + P];
  S T = temperature(p, x, nstep, st.shift);
  S h[NP], dh[NP * NP];
  interp_h(N, phiP, h, dh);
  S ps[NP];
  for (int b = 0; b < N; ++b) ps[b] = psi(p, b, mu, T);
  for (int al = 0; al < N; ++al) {
    S cell = 0;
    for (int be = 0; be < N; ++be) {
      if (be == al) continue;
      S q[3], dA[3];
      for (int e = 0; e < d; ++e) q[e] = phiP[al] * gc[be][e] - phiP[be] * gc[al][e];
      aniso_dAdq(d, q, p.gamma[al][be], p.delta[al][be], dA);
      for (int e = 0; e < d; ++e) cell += dA[e] * gc[be][e];
    }
    /* dW/dphi_a: obstacle (16/pi^2) sum_b gamma_ab phi_b (Eq. Wpot);
     * test-only well W = 9 sum_{a<b} gamma phi_a^2 phi_b^2 */
    S dW = 0;
    for (int be = 0; be < N; ++be) {
      if (be == al) continue;
      if (p.potential == GPFO_OBSTACLE)
        dW += S(16.0 / (PI * PI)) * p.gamma[al][be] * phiP[be];
      else
        dW += S(18.0) * p.gamma[al][be] * phiP[al] * phiP[be] * phiP[be];
    }
    S drive = 0; /* d Psi / d phi_a with Psi = sum_b psi^b h_b */
    for (int be = 0; be < N; ++be) drive += ps[be] * dh[be * N + al];
    R[al] = p.eps * (div[al] - cell) - dW / p.eps - drive;
  }
}

/* ---------------- S4: chemical potential ----------------------------------- */
/* Eq. (conc) in flux form, with C^a affine in mu and T:
 *   chi_tot = sum_a h_a(phi^{n+1}) chi,   c*(P) = sum_a h_a(phi^{n+1}) C^a(mu^n, T^n),
 *   M(P) = sum_a phi^{n+1}_a diag(D_a) chi,
 *   face P|Q:  J = -(M_P + M_Q)/2 (mu_Q - mu_P)/dx
 *                  + (U_P + U_Q)_a/2 (dx/dt) (c*_P + c*_Q)/2      (0 on walls)
 *   Delta = -dt div J - sum_a C^a(mu^n, T^n) (h_a^{n+1} - h_a^n)
 *           - sum_a h_a^{n+1} (C^a(mu^n, T^{n+1}) - C^a(mu^n, T^n))
 *   mu^{n+1} = mu^n + chi_tot^{-1} Delta.
 * The last term is the dT/dt term of Eq. (conc) over one step; with C^a
 * affine in mu it makes sum_a h_a C^a(mu, T) change exactly by -dt div J.
 * U is the lattice velocity of the previous step (U = 0 in solid cells),
 * converted to phase-field units by dx/dt (one LBM step per PF step). */
template <class S>
void mu_cell(const Grid& g, const Par<S>& p, const State<S>& st, const std::vector<S>& phin,
             const long* x, S* mu_new) {
  const int d = p.dim, N = p.N, nc = p.nc;
  const long cells = g.cells();
  auto cell_quant = [&](long j, S* M /*nc*nc*/, S* cstar /*nc*/) {
    S ph[NP] = {}, h[NP], dh[NP * NP];
    for (int a = 0; a < N; ++a) ph[a] = phin[a * cells + j];
    interp_h(N, ph, h, dh);
    S mu[2];
    for (int i = 0; i < nc; ++i) mu[i] = st.mu[i * cells + j];
    long xj[3];
    g.coords(j, xj);
    const S Tj = temperature(p, xj, st.step, st.shift);
    for (int i = 0; i < nc; ++i) {
      cstar[i] = 0;
      for (int k = 0; k < nc; ++k) M[i * nc + k] = 0;
    }
    for (int a = 0; a < N; ++a) {
      S C[2];
      comp_C(p, a, mu, Tj, C);
      for (int i = 0; i < nc; ++i) {
        cstar[i] += h[a] * C[i];
        for (int k = 0; k < nc; ++k) M[i * nc + k] += ph[a] * p.D[a][i] * p.chi[i][k];
      }
    }
  };
  const long P = g.idx(x[0], x[1], x[2]);
  S MP[4], cP[2];
  cell_quant(P, MP, cP);
  S divJ[2] = {0, 0};
  for (int a = 0; a < d; ++a) {
    for (int s = -1; s <= 1; s += 2) {
      long xq = x[a] + s;
      if (!p.periodic[a] && (xq < 0 || xq >= g.n[a])) continue;
      int off[3] = {0, 0, 0};
      off[a] = s;
      long Qi = g.field_nb(x, off);
      S MQ[4], cQ[2];
      cell_quant(Qi, MQ, cQ);
      S uf = S(0.5) * (st.u[a * cells + P] + st.u[a * cells + Qi]) * (p.dx / p.dt);
      for (int i = 0; i < nc; ++i) {
        /* flux in the +e_a direction through the face */
        S dmu_pos[2];
        for (int k = 0; k < nc; ++k)
          dmu_pos[k] = S((double)s) * (st.mu[k * cells + Qi] - st.mu[k * cells + P]) / p.dx;
        S JD = 0;
        for (int k = 0; k < nc; ++k) JD += -S(0.5) * (MP[i * nc + k] + MQ[i * nc + k]) * dmu_pos[k];
        S JA = uf * S(0.5) * (cP[i] + cQ[i]);
        divJ[i] += S((double)s) * (JD + JA) / p.dx;
      }
    }
  }
  S ph0[NP], ph1[NP], h0[NP], h1[NP], dh[NP * NP], mu[2];
  for (int a = 0; a < N; ++a) {
    ph0[a] = st.phi[a * cells + P];
    ph1[a] = phin[a * cells + P];
  }
  interp_h(N, ph0, h0, dh);
  interp_h(N, ph1, h1, dh);
  for (int i = 0; i < nc; ++i) mu[i] = st.mu[i * cells + P];
  const S T0 = temperature(p, x, st.step, st.shift), T1 = temperature(p, x, st.step + 1, st.shift);
  S Delta[2];
  for (int i = 0; i < nc; ++i) Delta[i] = -p.dt * divJ[i];
  for (int a = 0; a < N; ++a) {
    S C[2], C1[2];
    comp_C(p, a, mu, T0, C);
    comp_C(p, a, mu, T1, C1);
    for (int i = 0; i < nc; ++i) Delta[i] -= C[i] * (h1[a] - h0[a]);
    for (int i = 0; i < nc; ++i) Delta[i] -= h1[a] * (C1[i] - C[i]);
  }
  S sh = 0;
  for (int a = 0; a < N; ++a) sh += h1[a];
  if (nc == 1) {
    S chit = sh * p.chi[0][0];
    mu_new[0] = mu[0] + Delta[0] / chit;
  } else {
    S a11 = sh * p.chi[0][0], a12 = sh * p.chi[0][1], a21 = sh * p.chi[1][0],
      a22 = sh * p.chi[1][1];
    S det = a11 * a22 - a12 * a21;
    mu_new[0] = mu[0] + (a22 * Delta[0] - a12 * Delta[1]) / det;
    mu_new[1] = mu[1] + (-a21 * Delta[0] + a11 * Delta[1]) / det;
  }
}

/* ---------------- S5: forces, moments, BGK collision ------------------------ */
/* Shrinkage force (Eq. shrinkage): G_S = sum_a eta_a (dphi_a/dt) n_a with
 * eta_a = (rho_a - rho_liq)/rho_liq and n_a = grad phi_a / |grad phi_a|.
 * Reading: dphi/dt over one lattice time step (one LBM step per PF step), so
 * dphi_a/dt = phi^{n+1}_a - phi^n_a in lattice units; the normal from central
 * differences of phi^{n+1} (walls mirrored, periodic axes wrapped); n_a = 0
 * where |grad phi_a|^2 <= 1e-24. */
template <class S>
void shrinkage_force(const Grid& g, const Par<S>& p, const std::vector<S>& phi_old,
                     const std::vector<S>& phi_new, const long* x, S* GS) {
  const long cells = g.cells();
  const long P = g.idx(x[0], x[1], x[2]);
  for (int a = 0; a < 3; ++a) GS[a] = S(0.0);
  for (int b = 0; b < p.N; ++b) {
    if (p.eta[b] == S(0.0)) continue;
    S grad[3] = {0, 0, 0}, gg = 0;
    for (int a = 0; a < p.dim; ++a) {
      int op[3] = {0, 0, 0}, om[3] = {0, 0, 0};
      op[a] = 1;
      om[a] = -1;
      grad[a] = (phi_new[b * cells + g.field_nb(x, op)] - phi_new[b * cells + g.field_nb(x, om)]) /
                (S(2.0) * p.dx);
      gg += grad[a] * grad[a];
    }
    if (re(gg) <= 1e-24) continue;
    S rate = p.eta[b] * (phi_new[b * cells + P] - phi_old[b * cells + P]) / std::sqrt(gg);
    for (int a = 0; a < p.dim; ++a) GS[a] += rate * grad[a];
  }
}

/* rho = sum f, m = sum f c (Eq. rhovel);
 * buoyancy F_B = -rho phi_l sum_i gbeta_i (C^l_i(mu^{n+1}) - C_ref_i) g_hat (Eq. buoyancy,
 *   g_hat the unit gravity vector, gbeta the signed product g beta_i);
 * shrinkage G_S as above; explicit force F_E = F_B + G_S;
 * drag G_D = -kappa rho (1 - phi_l)^2 U, kappa = 2 nu h / W0, nu = (tau - 1/2)/3;
 * velocity with Guo's half-force correction, the drag taken implicitly:
 *   U = (m + F_E/2) / (rho (1 + kappa (1 - phi_l)^2 / 2)),  U = 0 where phi_l = 0;
 * F = F_E + G_D;  f* = f - (f - f^eq)/tau + Guo source. */
template <class S>
void collide_cell(const Lattice& L, const Par<S>& p, const S* fin, S phil,
                  const S* mu_new, S T1, const S* GS, S* fout, S* u_out) {
  const int d = p.dim;
  S rho = 0, m[3] = {0, 0, 0};
  for (int k = 0; k < L.Q; ++k) {
    rho += fin[k];
    for (int a = 0; a < d; ++a) m[a] += fin[k] * S((double)L.c[k][a]);
  }
  S Cl[2];
  comp_C(p, p.N - 1, mu_new, T1, Cl);
  S b = 0;
  for (int i = 0; i < p.nc; ++i) b += p.gbeta[i] * (Cl[i] - p.c_ref[i]);
  S FB[3] = {0, 0, 0};
  FB[p.grav_axis] = -rho * phil * b * S((double)p.grav_sign);
  for (int a = 0; a < d; ++a) FB[a] += GS[a];
  S nu = (p.tau_lb - S(0.5)) / S(3.0);
  S kappa = S(2.0) * nu * p.h_drag / p.W0;
  S sol = (S(1.0) - phil) * (S(1.0) - phil);
  S u[3] = {0, 0, 0}, F[3] = {0, 0, 0};
  if (re(phil) != 0.0) {
    for (int a = 0; a < d; ++a)
      u[a] = (m[a] + S(0.5) * FB[a]) / (rho * (S(1.0) + S(0.5) * kappa * sol));
  }
  for (int a = 0; a < d; ++a) F[a] = FB[a] - kappa * rho * sol * u[a];
  for (int k = 0; k < L.Q; ++k) {
    S fe = feq(L, k, rho, u, d);
    fout[k] = fin[k] - (fin[k] - fe) / p.tau_lb + guo(L, k, p.tau_lb, u, F, d);
  }
  for (int a = 0; a < d; ++a) u_out[a] = u[a];
}

/* ---------------- one coupled step ------------------------------------------- */

template <class S>
void step_once(const Grid& g, const Lattice& L, const Par<S>& p, State<S>& st) {
  const long cells = g.cells();
  const int N = p.N, nc = p.nc, d = p.dim, Q = L.Q;
  std::vector<S> phin(st.phi.size()), mun(st.mu.size()), fpost(st.f.size()),
      un(st.u.size()), fnew(st.f.size());
  const S rate = p.dt / (p.tau_pf * p.eps);

  /* S1-S3: phase field, phi^n and mu^n in, phi^{n+1} out */
#pragma omp parallel for schedule(static)
  for (long P = 0; P < cells; ++P) {
    long x[3];
    g.coords(P, x);
    unsigned A = active_set(g, L, p, st, x);
    int na = 0;
    for (int a = 0; a < N; ++a) na += (A >> a) & 1u;
    if (na <= 1) {
      for (int a = 0; a < N; ++a) phin[a * cells + P] = st.phi[a * cells + P];
      continue;
    }
    S R[NP];
    pf_rhs(g, p, st, x, st.step, R);
    S v[NP], w[NP];
    int m = 0;
    int which[NP];
    for (int a = 0; a < N; ++a)
      if ((A >> a) & 1u) {
        v[m] = st.phi[a * cells + P] + rate * R[a];
        which[m++] = a;
      }
    project_simplex(m, v, w);
    for (int a = 0; a < N; ++a) phin[a * cells + P] = S(0.0);
    for (int j = 0; j < m; ++j) phin[which[j] * cells + P] = w[j];
  }

  /* S4: chemical potential, phi^n, phi^{n+1}, mu^n, U^{n-1} in */
#pragma omp parallel for schedule(static)
  for (long P = 0; P < cells; ++P) {
    long x[3];
    g.coords(P, x);
    S mnew[2];
    mu_cell(g, p, st, phin, x, mnew);
    for (int i = 0; i < nc; ++i) mun[i * cells + P] = mnew[i];
  }

  /* S5: collision at every cell with phi^{n+1}_l and mu^{n+1} */
#pragma omp parallel for schedule(static)
  for (long P = 0; P < cells; ++P) {
    S fin[27], fo[27], uo[3], mnew[2], GS[3];
    long x[3];
    g.coords(P, x);
    shrinkage_force(g, p, st.phi, phin, x, GS);
    for (int k = 0; k < Q; ++k) fin[k] = st.f[k * cells + P];
    for (int i = 0; i < nc; ++i) mnew[i] = mun[i * cells + P];
    collide_cell(L, p, fin, phin[(N - 1) * cells + P], mnew, temperature(p, x, st.step + 1, st.shift), GS, fo,
                 uo);
    for (int k = 0; k < Q; ++k) fpost[k * cells + P] = fo[k];
    for (int a = 0; a < d; ++a) un[a * cells + P] = uo[a];
  }

  /* S6: pull streaming; populations that would come from outside a wall are
   * the reflected ones of the cell itself (half-way bounce-back, the wall on
   * the same face as the zero-flux faces of phi and mu).  Test-only moving
   * lid on the upper wall of axis 1: + 6 w_k rho0 c_k . U_wall. */
#pragma omp parallel for schedule(static)
  for (long P = 0; P < cells; ++P) {
    long x[3];
    g.coords(P, x);
    for (int k = 0; k < Q; ++k) {
      int off[3] = {-L.c[k][0], -L.c[k][1], -L.c[k][2]};
      long y[3];
      if (g.inside(x, off, y)) {
        fnew[k * cells + P] = fpost[k * cells + g.idx(y[0], y[1], y[2])];
      } else {
        S val = fpost[L.opp[k] * cells + P];
        if (x[1] - L.c[k][1] >= g.n[1] && !p.periodic[1])
          val += S(6.0) * L.w[k] * p.rho0 * S((double)L.c[k][0]) * p.lid_u;
        fnew[k * cells + P] = val;
      }
    }
  }

  st.phi.swap(phin);
  st.mu.swap(mun);
  st.f.swap(fnew);
  st.u.swap(un);
  st.step += 1;
}

/* ---------------- moving frame (Case 2: "a moving frame approach to follow
 * the growth front"; the paper gives no details) ------------------------------
 * Reading: after every frame_every steps the front is the largest pull-axis
 * index of a cell whose liquid fraction is at most 1/2; when it lies beyond
 * frame_front, every field (phi, mu, U, the stored populations) moves down the
 * pull axis by d = front - frame_front cells, the d new planes at the far end
 * repeat the last plane (zero gradient into the melt), the planes leaving at
 * the near end are dropped, and the frame origin `shift` grows by d (it
 * enters the frozen temperature). */
template <class S>
void frame_shift(const Grid& g, const Par<S>& p, State<S>& st) {
  if (p.frame_every <= 0 || st.step % p.frame_every != 0) return;
  const long cells = g.cells();
  const int ax = p.pull_axis;
  long front = -1;
  for (long P = 0; P < cells; ++P) {
    long x[3];
    g.coords(P, x);
    if (re(st.phi[(p.N - 1) * cells + P]) <= 0.5 && x[ax] > front) front = x[ax];
  }
  const long d = front - p.frame_front;
  if (front < 0 || d <= 0) return;
  auto move = [&](std::vector<S>& v) {
    const long ncomp = (long)v.size() / cells;
    std::vector<S> out(v.size());
    for (long c = 0; c < ncomp; ++c)
      for (long P = 0; P < cells; ++P) {
        long x[3];
        g.coords(P, x);
        long y[3] = {x[0], x[1], x[2]};
        y[ax] = std::min(x[ax] + d, g.n[ax] - 1);
        out[c * cells + P] = v[c * cells + g.idx(y[0], y[1], y[2])];
      }
    v.swap(out);
  };
  move(st.phi);
  move(st.mu);
  move(st.u);
  move(st.f);
  st.shift += d;
}

template <class S>
void advance(const Grid& g, const Lattice& L, const Par<S>& p, State<S>& st, int64_t nsteps) {
  for (int64_t i = 0; i < nsteps; ++i) {
    step_once(g, L, p, st);
    frame_shift(g, p, st);
  }
}

/* ---------------- initial state --------------------------------------------- */

/* SplitMix64 (Steele, Lea and Flood 2014) used as a counter-based generator:
 * output j = mix(seed + (j + 1) * 0x9E3779B97F4A7C15). */
uint64_t splitmix64(uint64_t seed, uint64_t j) {
  uint64_t z = seed + (j + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* standard normal number j of the stream: Box-Muller (1958) on the uniforms
 * of counters 2j and 2j+1, 53-bit, u1 in (0, 1] */
double normal_j(uint64_t seed, uint64_t j) {
  double u1 = ((double)(splitmix64(seed, 2 * j) >> 11) + 1.0) * (1.0 / 9007199254740992.0);
  double u2 = (double)(splitmix64(seed, 2 * j + 1) >> 11) * (1.0 / 9007199254740992.0);
  return std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * PI * u2);
}

/* solid fraction of the 1D equilibrium profile of the double obstacle
 * (from 2 gamma eps phi'' = dW/dphi / eps): 1/2 - 1/2 sin(4 s / (pi eps))
 * for |s| <= pi^2 eps / 8, where s is the signed distance from the interface
 * centre (positive on the liquid side). */
double obstacle_profile(double s, double eps) {
  double half = PI * PI * eps / 8.0;
  if (s <= -half) return 1.0;
  if (s >= half) return 0.0;
  return 0.5 - 0.5 * std::sin(4.0 * s / (PI * eps));
}

void init_state(gpfo_sim* S_, uint64_t seed) {
  const gpfo_params& p = S_->prm;
  const Grid& g = S_->g;
  const long cells = g.cells();
  State<double>& st = S_->st;
  st.phi.assign((size_t)p.N * cells, 0.0);
  st.mu.assign((size_t)p.nc * cells, 0.0);
  st.f.assign((size_t)S_->L.Q * cells, 0.0);
  st.u.assign((size_t)p.dim * cells, 0.0);
  st.step = 0;
  for (long P = 0; P < cells; ++P) {
    long x[3];
    g.coords(P, x);
    double sol = 0.0;
    int solid_phase = 0;
    if (p.init_kind == GPFO_INIT_SEED) {
      double r2 = 0;
      for (int a = 0; a < p.dim; ++a) {
        double dd = ((double)x[a] - p.init_center[a]) * p.dx;
        r2 += dd * dd;
      }
      sol = obstacle_profile(std::sqrt(r2) - p.init_radius * p.dx, p.eps);
    } else if (p.init_kind == GPFO_INIT_LAMELLAE) {
      double s = ((double)x[p.pull_axis] - p.lam_height) * p.dx;
      sol = obstacle_profile(s, p.eps);
      /* the N - 1 solids take turns along x, lam_width cells each */
      if (p.N >= 3 && p.lam_width > 0)
        solid_phase = ((long)std::floor((double)x[0] / p.lam_width)) % (p.N - 1);
    }
    st.phi[(size_t)solid_phase * cells + P] = sol;
    st.phi[(size_t)(p.N - 1) * cells + P] = 1.0 - sol;
    for (int i = 0; i < p.nc; ++i)
      st.mu[(size_t)i * cells + P] =
          p.mu_inf[i] + p.noise_sigma * normal_j(seed, (uint64_t)P * p.nc + i);
    for (int k = 0; k < S_->L.Q; ++k) st.f[(size_t)k * cells + P] = S_->L.w[k] * p.rho0;
  }
}

template <class S>
State<S> lift_state(const State<double>& s) {
  State<S> r;
  r.phi.assign(s.phi.begin(), s.phi.end());
  r.mu.assign(s.mu.begin(), s.mu.end());
  r.f.assign(s.f.begin(), s.f.end());
  r.u.assign(s.u.begin(), s.u.end());
  r.step = s.step;
  r.shift = s.shift;
  return r;
}

/* compensated (Neumaier) sum, so the oracle's totals carry no summation error
 * that would hide the conservation the method guarantees */
struct KSum {
  double s = 0, c = 0;
  void add(double v) {
    double t = s + v;
    if (std::fabs(s) >= std::fabs(v))
      c += (s - t) + v;
    else
      c += (v - t) + s;
    s = t;
  }
  double get() const { return s + c; }
};

}  // namespace

/* ============================ C interface ==================================== */

extern "C" {

gpfo_sim* gpfo_create(const gpfo_params* p, uint64_t seed) {
  if (!p) return nullptr;
  if (p->dim != 2 && p->dim != 3) return nullptr;
  if (p->N < 2 || p->N > NP || p->nc < 1 || p->nc > 2) return nullptr;
  gpfo_sim* s = new gpfo_sim;
  s->prm = *p;
  s->g.dim = p->dim;
  for (int a = 0; a < 3; ++a) {
    s->g.n[a] = (a < p->dim) ? (long)p->n[a] : 1;
    s->g.periodic[a] = (a < p->dim) ? p->periodic[a] : 1;
    if (s->g.n[a] < 1) {
      delete s;
      return nullptr;
    }
  }
  s->prm.periodic[2] = s->g.periodic[2];
  if (p->dim == 2) s->prm.n[2] = 1;
  s->L = (p->dim == 3 && p->lattice_q == 27) ? make_lattice_q(27) : make_lattice(p->dim);
  init_state(s, seed);
  return s;
}

void gpfo_destroy(gpfo_sim* s) { delete s; }

void gpfo_set_threads(int nthreads) {
#ifdef _OPENMP
  omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
}

void gpfo_step(gpfo_sim* s, int64_t nsteps) {
  Par<double> p = lift<double>(s->prm);
  advance(s->g, s->L, p, s->st, nsteps);
}

int64_t gpfo_step_index(const gpfo_sim* s) { return s->st.step; }
int64_t gpfo_frame_offset(const gpfo_sim* s) { return s->st.shift; }
int64_t gpfo_cells(const gpfo_sim* s) { return s->g.cells(); }
int32_t gpfo_Q(const gpfo_sim* s) { return s->L.Q; }

int64_t gpfo_field_count(const gpfo_sim* s, int32_t field) {
  long c = s->g.cells();
  switch (field) {
    case 0: return (int64_t)s->prm.N * c;
    case 1: return (int64_t)s->prm.nc * c;
    case 2: return (int64_t)s->L.Q * c;
    case 3: return c;
    case 4: return (int64_t)s->prm.dim * c;
    case 5: return (int64_t)s->prm.nc * c;
    case 6: return c;
    case 7: return c;
  }
  return -1;
}

int gpfo_get(const gpfo_sim* s, int32_t field, double* dst) {
  const long cells = s->g.cells();
  const State<double>& st = s->st;
  Par<double> p = lift<double>(s->prm);
  switch (field) {
    case 0: std::copy(st.phi.begin(), st.phi.end(), dst); return 0;
    case 1: std::copy(st.mu.begin(), st.mu.end(), dst); return 0;
    case 2: std::copy(st.f.begin(), st.f.end(), dst); return 0;
    case 3:
      for (long P = 0; P < cells; ++P) {
        double r = 0;
        for (int k = 0; k < s->L.Q; ++k) r += st.f[k * cells + P];
        dst[P] = r;
      }
      return 0;
    case 4: std::copy(st.u.begin(), st.u.end(), dst); return 0;
    case 5:
      for (long P = 0; P < cells; ++P) {
        double ph[NP], h[NP], dh[NP * NP], mu[2];
        for (int a = 0; a < p.N; ++a) ph[a] = st.phi[a * cells + P];
        for (int i = 0; i < p.nc; ++i) mu[i] = st.mu[i * cells + P];
        interp_h(p.N, ph, h, dh);
        long x[3];
        s->g.coords(P, x);
        const double T = temperature(p, x, st.step, st.shift);
        for (int i = 0; i < p.nc; ++i) dst[i * cells + P] = 0;
        for (int a = 0; a < p.N; ++a) {
          double C[2];
          comp_C(p, a, mu, T, C);
          for (int i = 0; i < p.nc; ++i) dst[i * cells + P] += h[a] * C[i];
        }
      }
      return 0;
    case 6:
      for (long P = 0; P < cells; ++P) {
        long x[3];
        s->g.coords(P, x);
        dst[P] = temperature(p, x, st.step, st.shift);
      }
      return 0;
    case 7:
      for (long P = 0; P < cells; ++P) {
        long x[3];
        s->g.coords(P, x);
        dst[P] = (double)active_set(s->g, s->L, p, st, x);
      }
      return 0;
  }
  return -1;
}

int gpfo_set(gpfo_sim* s, int32_t field, const double* src) {
  State<double>& st = s->st;
  switch (field) {
    case 0: std::copy(src, src + st.phi.size(), st.phi.begin()); return 0;
    case 1: std::copy(src, src + st.mu.size(), st.mu.begin()); return 0;
    case 2: std::copy(src, src + st.f.size(), st.f.begin()); return 0;
    case 4: std::copy(src, src + st.u.size(), st.u.begin()); return 0;
  }
  return -1;
}

int gpfo_total(const gpfo_sim* s, int32_t which, double* out) {
  const long cells = s->g.cells();
  if (which == 0) {
    std::vector<double> C((size_t)s->prm.nc * cells);
    gpfo_get(s, 5, C.data());
    for (int i = 0; i < s->prm.nc; ++i) {
      KSum k;
      for (long P = 0; P < cells; ++P) k.add(C[i * cells + P]);
      out[i] = k.get();
    }
    return 0;
  }
  if (which == 1) {
    KSum k;
    for (size_t j = 0; j < s->st.f.size(); ++j) k.add(s->st.f[j]);
    out[0] = k.get();
    return 0;
  }
  return -1;
}

int gpfo_lattice(int32_t Q, int32_t* c_out, double* w_out, int32_t* opp_out) {
  if (Q != 9 && Q != 19 && Q != 27) return -1;
  Lattice L = make_lattice_q(Q);
  for (int k = 0; k < L.Q; ++k) {
    for (int a = 0; a < 3; ++a) c_out[3 * k + a] = L.c[k][a];
    w_out[k] = L.w[k];
    opp_out[k] = L.opp[k];
  }
  return L.Q;
}

double gpfo_aniso_ac(int32_t dim, const double* q, double delta) { return aniso_ac(dim, q, delta); }
double gpfo_aniso_A(int32_t dim, const double* q, double gamma, double delta) {
  return aniso_A(dim, q, gamma, delta);
}
void gpfo_aniso_dAdq(int32_t dim, const double* q, double gamma, double delta, double* out) {
  aniso_dAdq(dim, q, gamma, delta, out);
}
void gpfo_aniso_dAdq_cs(int32_t dim, const double* q, double gamma, double delta, double h,
                        double* out) {
  for (int a = 0; a < dim; ++a) {
    cplx qc[3];
    for (int b = 0; b < dim; ++b) qc[b] = cplx(q[b], b == a ? h : 0.0);
    cplx A = aniso_A<cplx>(dim, qc, cplx(gamma), cplx(delta));
    out[a] = A.imag() / h;
  }
}
int gpfo_project(int32_t m, const double* v, double* out) {
  if (m < 1) return -1;
  project_simplex(m, v, out);
  return 0;
}
void gpfo_interp_h(int32_t N, const double* phi, double* h, double* dh) { interp_h(N, phi, h, dh); }
void gpfo_feq(int32_t Q, double rho, const double* u, double* out) {
  Lattice L = make_lattice_q(Q);
  const int dim = Q == 9 ? 2 : 3;
  for (int k = 0; k < L.Q; ++k) out[k] = feq(L, k, rho, u, dim);
}
void gpfo_guo(int32_t Q, double tau, const double* u, const double* F, double* S) {
  Lattice L = make_lattice_q(Q);
  const int dim = Q == 9 ? 2 : 3;
  for (int k = 0; k < L.Q; ++k) S[k] = guo(L, k, tau, u, F, dim);
}
double gpfo_normal(uint64_t seed, uint64_t j) { return normal_j(seed, j); }

int gpfo_grand_potential(const gpfo_params* prm, int32_t a, const double* mu, double T, double h,
                         double* psi_out, double* dpsi_dmu, double* dpsi_dT, double* conc) {
  if (!prm || a < 0 || a >= prm->N || prm->nc < 1 || prm->nc > 2 || !(h > 0)) return -1;
  const Par<double> pd = lift<double>(*prm);
  const Par<cplx> pc = lift<cplx>(*prm);
  *psi_out = psi(pd, a, mu, T);
  for (int i = 0; i < prm->nc; ++i) {
    cplx m[2];
    for (int j = 0; j < prm->nc; ++j) m[j] = cplx(mu[j], j == i ? h : 0.0);
    dpsi_dmu[i] = psi(pc, a, m, cplx(T)).imag() / h;
  }
  cplx m[2];
  for (int j = 0; j < prm->nc; ++j) m[j] = cplx(mu[j]);
  *dpsi_dT = psi(pc, a, m, cplx(T, h)).imag() / h;
  comp_C(pd, a, mu, T, conc);
  return 0;
}

int gpfo_loss_grad_cs(const gpfo_sim* s, int64_t nsteps, const double* target, int32_t which,
                      double h, double* loss_out, double* grad_out) {
  Par<cplx> p = lift<cplx>(s->prm);
  const cplx ih(0.0, h);
  switch (which) {
    case GPFO_P_DELTA:
      for (int a = 0; a < NP; ++a)
        for (int b = 0; b < NP; ++b)
          if (s->prm.delta[a][b] != 0.0) p.delta[a][b] += ih;
      break;
    case GPFO_P_TAU: p.tau_pf += ih; break;
    case GPFO_P_DIFF: p.D[s->prm.N - 1][0] += ih; break;
    case GPFO_P_GBETA: p.gbeta[0] += ih; break;
    case GPFO_P_DIFF1: p.D[s->prm.N - 1][1] += ih; break;
    case GPFO_P_GBETA1: p.gbeta[1] += ih; break;
    default: return -1;
  }
  State<cplx> st = lift_state<cplx>(s->st);
  advance(s->g, s->L, p, st, nsteps);
  cplx L = 0;
  for (size_t j = 0; j < st.phi.size(); ++j) {
    cplx e = st.phi[j] - target[j];
    L += 0.5 * e * e;
  }
  if (loss_out) *loss_out = L.real();
  if (grad_out) *grad_out = L.imag() / h;
  return 0;
}

int gpfo_tangent_cs(const gpfo_sim* s, int64_t nsteps, int32_t field, const double* dir, double h,
                    int32_t out_field, double* out) {
  Par<cplx> p = lift<cplx>(s->prm);
  State<cplx> st = lift_state<cplx>(s->st);
  std::vector<cplx>* v = nullptr;
  switch (field) {
    case 0: v = &st.phi; break;
    case 1: v = &st.mu; break;
    case 2: v = &st.f; break;
    case 4: v = &st.u; break;
    default: return -1;
  }
  for (size_t j = 0; j < v->size(); ++j) (*v)[j] += cplx(0.0, h * dir[j]);
  advance(s->g, s->L, p, st, nsteps);
  std::vector<cplx>* o = nullptr;
  switch (out_field) {
    case 0: o = &st.phi; break;
    case 1: o = &st.mu; break;
    case 2: o = &st.f; break;
    case 4: o = &st.u; break;
    default: return -1;
  }
  for (size_t j = 0; j < o->size(); ++j) out[j] = (*o)[j].imag() / h;
  return 0;
}

}  // extern "C"
