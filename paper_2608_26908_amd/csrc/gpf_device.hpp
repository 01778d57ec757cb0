// gpf_device.hpp -- device-side building blocks of the coupled GP
// phase-field / lattice-Boltzmann step for gfx950: lattice tables, the
// per-launch parameter block and the pointwise model functions.
//
// Storage precision R is float or double; arithmetic is carried out in R.
// Every field is structure-of-arrays [component][z][y][x], x fastest.
#pragma once
#include <type_traits>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gpf {

// ---------------------------------------------------------------------------
// Lattices.  D2Q9 numbering of the paper's lattice figure with the weights of
// Table LBM_Schemes; D3Q19 is the textbook 19-velocity set (the paper's own
// 3D lattice is D3Q27).  The neighbourhood a cell update reads is the same
// set of offsets, so one table serves the stencils and the streaming.
// ---------------------------------------------------------------------------
template <int Q> struct Lat;

template <> struct Lat<9> {
  static constexpr int Q = 9;
  __host__ __device__ static constexpr int c(int k, int a) {
    constexpr int t[9][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
                             {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
    return t[k][a];
  }
  __host__ __device__ static constexpr int opp(int k) {
    constexpr int t[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    return t[k];
  }
  __host__ __device__ static constexpr double w(int k) {
    return k == 0 ? 4.0 / 9.0 : (k <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
  }
};

template <> struct Lat<19> {
  static constexpr int Q = 19;
  __host__ __device__ static constexpr int c(int k, int a) {
    constexpr int t[19][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                              {0, 0, 1},  {0, 0, -1},  {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                              {-1, 1, 0}, {1, 0, 1},   {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                              {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
    return t[k][a];
  }
  __host__ __device__ static constexpr int opp(int k) {
    constexpr int t[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
    return t[k];
  }
  __host__ __device__ static constexpr double w(int k) {
    return k == 0 ? 1.0 / 3.0 : (k <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
  }
};

// D3Q27 of Table LBM_Schemes: the D3Q19 directions in the same order, then
// the 8 corners in opposite pairs; weights 8/27, 2/27, 1/54, 1/216
template <> struct Lat<27> {
  static constexpr int Q = 27;
  __host__ __device__ static constexpr int c(int k, int a) {
    constexpr int t[27][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                              {0, 0, 1},  {0, 0, -1},  {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                              {-1, 1, 0}, {1, 0, 1},   {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                              {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1},
                              {1, 1, 1},  {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1},
                              {1, -1, 1}, {-1, 1, -1}, {-1, 1, 1}, {1, -1, -1}};
    return t[k][a];
  }
  __host__ __device__ static constexpr int opp(int k) {
    constexpr int t[27] = {0,  2,  1,  4,  3,  6,  5,  8,  7,  10, 9,  12, 11, 14,
                           13, 16, 15, 18, 17, 20, 19, 22, 21, 24, 23, 26, 25};
    return t[k];
  }
  __host__ __device__ static constexpr double w(int k) {
    return k == 0 ? 8.0 / 27.0 : (k <= 6 ? 2.0 / 27.0 : (k <= 18 ? 1.0 / 54.0 : 1.0 / 216.0));
  }
};

// ---------------------------------------------------------------------------
// Parameters of one launch, passed by value (kernel arguments).
// ---------------------------------------------------------------------------
template <class R> struct KP {
  int n[3];
  int per[3];
  int64_t sy, sz, cells;  // strides of y and z, number of cells
  int potential;          // 0 obstacle, 1 well
  int pull_axis, grav_axis;
  R dx, dt, eps, rate;    // rate = dt / (tau_pf eps)
  R tau_pf;
  R gamma[4][4], delta[4][4];
  R chi[2][2], c0[4][2], dS[4];
  // chemical potentials are stored as mu - mu_ref (mu_ref = far-field mu in
  // FP32 storage, 0 in FP64), so C^a = c0s[a] + chi (mu - mu_ref)
  R mu_ref[2], c0s[4][2];
  double mu_ref_d[2], c0s_d[4][2];
  R D[4][2];
  R G, tdev_iso, T_E;     // T - T_E = G (x_pull - shift) if G != 0, else tdev_iso
  R mT[4][2];             // d c0_a / dT: C^a = c0s[a] + mT[a] (T - T_E) + chi (mu - mu_ref)
  R dtdev;                // T^{n+1} - T^n of one step, -G V (formed in FP64 on the host)
  int tdep;               // some mT != 0 (the compositions depend on T)
  R tau_lb, rho0, gbeta[2], c_ref[2], grav_sign, kappa, lid_u;
  // formed in FP64 on the host: 1 / tau_lb, the Guo prefactor 1 - 1 / (2 tau_lb),
  // 1 / dx, the lattice-to-phase-field velocity factor dx / dt and 1 / eps
  R omega, guo, idx, conv, ieps;
  R eta[4];               // shrinkage (rho_a - rho_liq) / rho_liq per phase
  int shrink;             // some eta != 0
  R qmin2;                // |q|^2 below which the anisotropy direction is undefined
  R w[27];                // lattice weights in R
};

// ---------------------------------------------------------------------------
// Pointwise model functions.
// ---------------------------------------------------------------------------

__device__ __forceinline__ float gsqrt(float v) { return sqrtf(v); }
__device__ __forceinline__ double gsqrt(double v) { return sqrt(v); }

// Forward-mode dual number: value and one directional derivative.  Used to
// differentiate dA/dq (Hessian-vector products and the derivative in delta)
// with the very code that evaluates it.
template <class R> struct Dual {
  R v, d;
  __device__ __forceinline__ Dual() : v(R(0)), d(R(0)) {}
  __device__ __forceinline__ Dual(R a) : v(a), d(R(0)) {}
  __device__ __forceinline__ Dual(R a, R b) : v(a), d(b) {}
};
template <class R> __device__ __forceinline__ Dual<R> operator+(Dual<R> a, Dual<R> b) { return {a.v + b.v, a.d + b.d}; }
template <class R> __device__ __forceinline__ Dual<R> operator-(Dual<R> a, Dual<R> b) { return {a.v - b.v, a.d - b.d}; }
template <class R> __device__ __forceinline__ Dual<R> operator*(Dual<R> a, Dual<R> b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
template <class R> __device__ __forceinline__ Dual<R> operator/(Dual<R> a, Dual<R> b) {
  const R q = a.v / b.v;
  return {q, (a.d - q * b.d) / b.v};
}
template <class R> __device__ __forceinline__ Dual<R>& operator+=(Dual<R>& a, Dual<R> b) { a = a + b; return a; }
template <class R> __device__ __forceinline__ R value_of(R x) { return x; }
template <class R> __device__ __forceinline__ R value_of(Dual<R> x) { return x.v; }

// dA/dq of the pair energy A(q) = gamma a_c(q)^2 |q|^2 with the cubic
// anisotropy a_c = 1 - delta (3 - 4 sum q_a^4 / |q|^4) (2D: 1 + delta cos 4theta):
//   dA/dq = 2 gamma a_c (a_c q + |q|^2 grad a_c),
//   grad a_c = 16 delta (q_a^3 / |q|^4 - q_a sum q^4 / |q|^6);
// a_c = 1 and grad a_c = 0 below |q|^2 = qmin2.  T is R or Dual<R>.
template <int D, class T, class R>
__device__ __forceinline__ void dAdq(const T (&q)[D], T gamma, T delta, R qmin2, T (&out)[D]) {
  if constexpr (std::is_same<T, R>::value) {
    // isotropic pair: the general expression reduces to 2 gamma q exactly
    if (delta == R(0)) {
#pragma unroll
      for (int a = 0; a < D; ++a) out[a] = R(2) * gamma * q[a];
      return;
    }
  }
  T q2 = T(R(0)), q4 = T(R(0));
#pragma unroll
  for (int a = 0; a < D; ++a) {
    T s = q[a] * q[a];
    q2 += s;
    q4 += s * s;
  }
  if (!(value_of(q2) > qmin2)) {
#pragma unroll
    for (int a = 0; a < D; ++a) out[a] = T(R(2)) * gamma * q[a];
    return;
  }
  T inv = T(R(1)) / q2;
  T inv2 = inv * inv;
  T ac = T(R(1)) - delta * (T(R(3)) - T(R(4)) * q4 * inv2);
#pragma unroll
  for (int a = 0; a < D; ++a) {
    T g = T(R(16)) * delta * inv2 * (q[a] * q[a] * q[a] - q[a] * q4 * inv);
    out[a] = T(R(2)) * gamma * ac * (ac * q[a] + q2 * g);
  }
}

// H(q) w (H = d^2 A / dq^2, symmetric) and d(dA/dq)/d delta . w, by forward
// mode through dAdq.
template <int D, class R>
__device__ __forceinline__ void dAdq_vjp(const R (&q)[D], R gamma, R delta, R qmin2, const R (&w)[D],
                                         R (&Hw)[D], R& ddelta_w) {
  if (delta == R(0)) {
    // isotropic pair: H = 2 gamma I exactly; the delta derivative is not
    // asked for pairs without anisotropy
#pragma unroll
    for (int a = 0; a < D; ++a) Hw[a] = R(2) * gamma * w[a];
    ddelta_w = R(0);
    return;
  }
  Dual<R> qd[D], out[D];
#pragma unroll
  for (int a = 0; a < D; ++a) qd[a] = Dual<R>(q[a], w[a]);
  dAdq<D, Dual<R>, R>(qd, Dual<R>(gamma), Dual<R>(delta), qmin2, out);
#pragma unroll
  for (int a = 0; a < D; ++a) {
    Hw[a] = out[a].d;
    qd[a] = Dual<R>(q[a]);
  }
  dAdq<D, Dual<R>, R>(qd, Dual<R>(gamma), Dual<R>(delta, R(1)), qmin2, out);
  ddelta_w = R(0);
#pragma unroll
  for (int a = 0; a < D; ++a) ddelta_w += out[a].d * w[a];
}

// Interpolation h_a(phi): phi_a^2 (3 - 2 phi_a), plus for N >= 3
// 2 phi_a e_a with e_a the sum over pairs of the other phases of their
// product (N = 3: the product of the other two, so 2 phi_0 phi_1 phi_2 for
// every phase).  Sum h = 1 on the simplex.
template <int N, class R>
__device__ __forceinline__ R pair_sum_others(const R (&ph)[N], int b) {
  R e = R(0);
#pragma unroll
  for (int g = 0; g < N; ++g)
#pragma unroll
    for (int k = g + 1; k < N; ++k)
      if (g != b && k != b) e += ph[g] * ph[k];
  return e;
}
template <int N, class R>
__device__ __forceinline__ void interp_h(const R (&ph)[N], R (&h)[N]) {
  if constexpr (N == 3) {
    const R tri = R(2) * ph[0] * ph[1] * ph[2];
#pragma unroll
    for (int b = 0; b < N; ++b) h[b] = ph[b] * ph[b] * (R(3) - R(2) * ph[b]) + tri;
  } else {
#pragma unroll
    for (int b = 0; b < N; ++b) {
      h[b] = ph[b] * ph[b] * (R(3) - R(2) * ph[b]);
      if (N >= 4) h[b] += R(2) * ph[b] * pair_sum_others<N, R>(ph, b);
    }
  }
}

// dh_b / dphi_a, a fixed.
template <int N, class R>
__device__ __forceinline__ R dh(const R (&ph)[N], int b, int a) {
  R r = (a == b) ? R(6) * ph[b] * (R(1) - ph[b]) : R(0);
  if constexpr (N == 3) {
    R other = R(1);
#pragma unroll
    for (int g = 0; g < N; ++g)
      if (g != a) other *= ph[g];
    r += R(2) * other;
  } else if constexpr (N >= 4) {
    if (a == b) {
      r += R(2) * pair_sum_others<N, R>(ph, b);
    } else {
      R rest = R(0);  // d e_b / d phi_a: the phases other than a and b
#pragma unroll
      for (int g = 0; g < N; ++g)
        if (g != a && g != b) rest += ph[g];
      r += R(2) * ph[b] * rest;
    }
  }
  return r;
}

// Euclidean projection onto the simplex {sum = 1, >= 0} of the entries of v
// selected by `mask` (the others are set to 0): sort the selected values
// descending, take the largest j with u_j - (sum_{i<=j} u_i - 1)/j > 0,
// theta = (sum_{i<=j} u_i - 1)/j, result max(v - theta, 0) (Held, Wolfe and
// Crowder 1974).  A sorting network on fixed-size arrays (3 or 4 slots),
// unselected entries sorted last.
template <int N, class R>
__device__ __forceinline__ void project_masked(unsigned mask, const R (&v)[N], R (&out)[N], R& theta) {
  constexpr int M = N > 3 ? N : 3;
  R u[M];
  bool on[M];
#pragma unroll
  for (int i = 0; i < M; ++i) {
    on[i] = (i < N) && ((mask >> i) & 1u);
    u[i] = (i < N) ? v[i] : R(0);
  }
  // descending by (selected, value)
  auto cs = [&](int i, int j) {
    const bool swap = (!on[i] && on[j]) || (on[i] == on[j] && u[j] > u[i]);
    if (swap) {
      R t = u[i]; u[i] = u[j]; u[j] = t;
      bool b = on[i]; on[i] = on[j]; on[j] = b;
    }
  };
  if constexpr (M == 3) {
    cs(0, 1);
    cs(1, 2);
    cs(0, 1);
  } else {
    cs(0, 1);
    cs(2, 3);
    cs(0, 2);
    cs(1, 3);
    cs(1, 2);
  }
  R csum = u[0];
  theta = u[0] - R(1);  // j = 1 always qualifies
#pragma unroll
  for (int j = 1; j < M; ++j) {
    if (on[j]) {
      csum += u[j];
      const R t = (csum - R(1)) / R(j + 1);
      if (u[j] - t > R(0)) theta = t;
    }
  }
#pragma unroll
  for (int i = 0; i < N; ++i)
    out[i] = (((mask >> i) & 1u) && v[i] - theta > R(0)) ? v[i] - theta : R(0);
}

// Neighbour coordinate along one axis for field values: periodic axes wrap,
// walls mirror the adjacent cell (zero normal derivative).
__device__ __forceinline__ int nb_field(int x, int s, int n, int per) {
  int y = x + s;
  if (y < 0) y = per ? y + n : 0;
  if (y >= n) y = per ? y - n : n - 1;
  return y;
}

}  // namespace gpf
