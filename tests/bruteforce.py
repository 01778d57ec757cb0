"""Literal, slow evaluator of one coupled step on tiny grids (pure Python
loops), written independently of the oracle to pin it by brute force.

Differences in route from the oracle, so that a slip in either shows up:
  * every derivative of an energy (dA/dq, dW/dphi, dPsi/dphi) is taken by
    complex step of the energy itself, not from a hand-derived formula;
  * the simplex projection enumerates all supports and keeps the one that
    satisfies the KKT conditions;
  * lattice vectors are generated from their definition (all vectors with
    components in {-1, 0, 1} and |c|^2 <= 1 in 2D-with-diagonals / <= 2 in 3D)
    and weights from the moment conditions, then re-ordered to the
    documented numbering;
  * fluxes are accumulated face by face over a list of faces, not per cell.
"""
import itertools
import math

import numpy as np

H_CS = 1e-30
PI = math.pi


def lattice(dim, kind=None):
    if kind == "D3Q27":
        # the paper's Table LBM_Schemes: rest 8/27, faces 2/27, edges 1/54,
        # corners 1/216; every velocity of {-1, 0, 1}^3, ordered by length
        c = sorted(itertools.product((-1, 0, 1), repeat=3), key=lambda v: sum(x * x for x in v))
        wmap = {0: 8 / 27, 1: 2 / 27, 2: 1 / 54, 3: 1 / 216}
        return c, [wmap[sum(x * x for x in v)] for v in c]
    if dim == 2:
        order = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
        c = [tuple(v) + (0,) for v in order]
        wmap = {0: 4 / 9, 1: 1 / 9, 2: 1 / 36}
    else:
        c = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
             (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1),
             (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]
        wmap = {0: 1 / 3, 1: 1 / 18, 2: 1 / 36}
    w = [wmap[sum(x * x for x in v)] for v in c]
    return c, w


def A_pair(q, gamma, delta):
    q2 = sum(x * x for x in q)
    if q2.real <= 1e-24:
        ac = 1.0
    else:
        ac = 1 - delta * (3 - 4 * sum(x ** 4 for x in q) / q2 ** 2)
    return gamma * ac * ac * q2


def dA_cs(q, gamma, delta):
    out = []
    for a in range(len(q)):
        qq = [complex(x) for x in q]
        qq[a] += 1j * H_CS
        out.append(A_pair(qq, gamma, delta).imag / H_CS)
    return out


def h_funcs(phi):
    N = len(phi)
    h = [p * p * (3 - 2 * p) for p in phi]
    if N >= 3:
        # + 2 phi_a times every product of two other phases
        for a in range(N):
            others = [phi[b] for b in range(N) if b != a]
            h[a] += 2 * phi[a] * sum(others[i] * others[j] for i in range(len(others))
                                     for j in range(i + 1, len(others)))
    return h


def grad_cs(fun, x):
    """complex-step gradient of a scalar function of a list of reals"""
    g = []
    for a in range(len(x)):
        xx = [complex(v) for v in x]
        xx[a] += 1j * H_CS
        g.append(fun(xx).imag / H_CS)
    return g


def project_kkt(v):
    m = len(v)
    for r in range(1, m + 1):
        for S in itertools.combinations(range(m), r):
            theta = (sum(v[i] for i in S) - 1) / r
            if all(v[i] - theta > 0 for i in S) and all(v[i] - theta <= 0 for i in range(m) if i not in S):
                return [v[i] - theta if i in S else 0.0 for i in range(m)]
    raise AssertionError("no KKT support")


class Step:
    """cfg: workload dict; state: dict of numpy arrays phi [N,...], mu [nc,...],
    f [Q,...], u [dim,...] in [comp][z][y][x] order (x fastest)."""

    def __init__(self, cfg):
        self.cfg = cfg
        self.dim = cfg["dim"]
        self.n = list(cfg["n"][: self.dim])
        self.per = list(cfg["periodic"][: self.dim])
        self.N, self.nc = cfg["N"], cfg["nc"]
        self.c, self.w = lattice(self.dim, cfg.get("lattice"))
        self.Q = len(self.c)

    # ----- index helpers (x = (x, y[, z]) tuple) -----
    def cells(self):
        return list(itertools.product(*[range(k) for k in self.n]))

    def at(self, arr, comp, x):
        return arr[(comp,) + tuple(reversed(x))]

    def wrap_field(self, x):
        y = list(x)
        for a in range(self.dim):
            if y[a] < 0:
                y[a] = y[a] + self.n[a] if self.per[a] else 0
            elif y[a] >= self.n[a]:
                y[a] = y[a] - self.n[a] if self.per[a] else self.n[a] - 1
        return tuple(y)

    def inside(self, x):
        y = list(x)
        for a in range(self.dim):
            if y[a] < 0 or y[a] >= self.n[a]:
                if not self.per[a]:
                    return None
                y[a] %= self.n[a]
        return tuple(y)

    def add(self, x, o):
        return tuple(x[a] + o[a] for a in range(self.dim))

    def phi(self, st, b, x):
        return self.at(st["phi"], b, self.wrap_field(x))

    def gradc(self, st, b, x, e):
        dx = self.cfg["dx"]
        ep = [0] * self.dim
        ep[e] = 1
        em = [0] * self.dim
        em[e] = -1
        return (self.phi(st, b, self.add(x, ep)) - self.phi(st, b, self.add(x, em))) / (2 * dx)

    def temperature(self, x, n):
        cf = self.cfg
        if cf["G"] == 0:
            return cf["T_iso"]
        return cf["T_E"] + cf["G"] * (x[cf["pull_axis"]] - cf["y0"] - cf["V"] * n)

    def c0T(self, a, T):
        """parabola centre of phase a at temperature T: c0 + mT (T - T_E)"""
        cf = self.cfg
        mT = np.array(cf.get("mT", [[0.0, 0.0]] * 4)[a][: self.nc], dtype=float)
        return np.array(cf["c0"][a][: self.nc]) + mT * (T - cf["T_E"])

    def psi(self, a, mu, T):
        cf = self.cfg
        chi = np.array(cf["chi"])[: self.nc, : self.nc]
        m = np.array(mu)
        return -0.5 * m @ chi @ m - m @ self.c0T(a, T) + cf["dS"][a] * (T - cf["T_E"])

    def C(self, a, mu, T):
        cf = self.cfg
        chi = np.array(cf["chi"])[: self.nc, : self.nc]
        return self.c0T(a, T) + chi @ np.array(mu)

    # ----- phase field -----
    def faces(self):
        """every interior face once: (P, Q, axis), Q = P + e_axis"""
        out = []
        for x in self.cells():
            for a in range(self.dim):
                o = [0] * self.dim
                o[a] = 1
                y = self.add(x, o)
                if y[a] >= self.n[a]:
                    if not self.per[a]:
                        continue
                    y = self.inside(y)
                out.append((x, y, a))
        return out

    def face_flux(self, st, x, y, a):
        """J_alpha (component a) on the face between x and y = x + e_a"""
        cf, N, d, dx = self.cfg, self.N, self.dim, self.cfg["dx"]
        ph = [0.5 * (self.phi(st, b, x) + self.phi(st, b, y)) for b in range(N)]
        gr = []
        for b in range(N):
            g = []
            for e in range(d):
                if e == a:
                    g.append((self.phi(st, b, y) - self.phi(st, b, x)) / dx)
                else:
                    g.append(0.5 * (self.gradc(st, b, x, e) + self.gradc(st, b, y, e)))
            gr.append(g)
        J = [0.0] * N
        for al in range(N):
            for be in range(N):
                if be == al:
                    continue
                q = [ph[al] * gr[be][e] - ph[be] * gr[al][e] for e in range(d)]
                dA = dA_cs(q, cf["gamma"][al][be], cf["delta"][al][be])
                J[al] += -ph[be] * dA[a]
        return J

    def pf(self, st):
        cf, N, d = self.cfg, self.N, self.dim
        eps, dx = cf["eps"], cf["dx"]
        div = {x: [0.0] * N for x in self.cells()}
        for (x, y, a) in self.faces():
            J = self.face_flux(st, x, y, a)
            for al in range(N):
                div[x][al] += J[al] / dx
                div[y][al] -= J[al] / dx
        new = np.array(st["phi"], dtype=float)
        # phase-field neighbourhood: the 9 / 19 points (no 3D corners)
        offs = [o[: d] for o in self.c if sum(1 for v in o if v) < 3]
        for x in self.cells():
            act = [b for b in range(N) if any(self.phi(st, b, self.add(x, o)) > 0 for o in offs)]
            if len(act) <= 1:
                continue
            phiP = [self.phi(st, b, x) for b in range(N)]
            gc = [[self.gradc(st, b, x, e) for e in range(d)] for b in range(N)]
            mu = [self.at(st["mu"], i, x) for i in range(self.nc)]
            T = self.temperature(x, st["step"])

            def energy_local(ph):
                """a(phi, grad phi) at the cell with grad phi frozen, plus W/eps^2
                and Psi/eps, so that -eps * d/dphi of it gives the local terms"""
                a_ = 0
                for al in range(N):
                    for be in range(al + 1, N):
                        q = [ph[al] * gc[be][e] - ph[be] * gc[al][e] for e in range(d)]
                        a_ += A_pair(q, cf["gamma"][al][be], cf["delta"][al][be])
                W = 0
                for al in range(N):
                    for be in range(al + 1, N):
                        if cf.get("potential", "obstacle") == "obstacle":
                            W += 16 / PI ** 2 * cf["gamma"][al][be] * ph[al] * ph[be]
                        else:
                            W += 9 * cf["gamma"][al][be] * ph[al] ** 2 * ph[be] ** 2
                hh = h_funcs(ph)
                Psi = sum(self.psi(b, mu, T) * hh[b] for b in range(N))
                return eps * a_ + W / eps + Psi

            g = grad_cs(energy_local, phiP)
            R = [eps * div[x][al] - g[al] for al in range(N)]
            rate = cf["dt"] / (cf["tau_pf"] * eps)
            v = [phiP[b] + rate * R[b] for b in act]
            pv = project_kkt(v)
            for b in range(N):
                new[(b,) + tuple(reversed(x))] = 0.0
            for j, b in enumerate(act):
                new[(b,) + tuple(reversed(x))] = pv[j]
        return new

    # ----- chemical potential -----
    def mu_update(self, st, phin):
        cf, N, nc, d, dx, dt = self.cfg, self.N, self.nc, self.dim, self.cfg["dx"], self.cfg["dt"]
        chi = np.array(cf["chi"])[:nc, :nc]

        n = st["step"]

        def quant(x):
            ph = [phin[(b,) + tuple(reversed(x))] for b in range(N)]
            hh = h_funcs(ph)
            mu = [self.at(st["mu"], i, x) for i in range(nc)]
            cs = sum(hh[b] * self.C(b, mu, self.temperature(x, n)) for b in range(N))
            M = sum(ph[b] * np.diag(cf["D"][b][:nc]) @ chi for b in range(N))
            return M, cs, np.array(mu)

        divJ = {x: np.zeros(nc) for x in self.cells()}
        for (x, y, a) in self.faces():
            Mx, cx, mx = quant(x)
            My, cy, my = quant(y)
            ux = self.at(st["u"], a, x)
            uy = self.at(st["u"], a, y)
            J = -0.5 * (Mx + My) @ (my - mx) / dx + 0.5 * (ux + uy) * dx / dt * 0.5 * (cx + cy)
            divJ[x] += J / dx
            divJ[y] -= J / dx
        new = np.array(st["mu"], dtype=float)
        for x in self.cells():
            ph0 = [self.at(st["phi"], b, x) for b in range(N)]
            ph1 = [phin[(b,) + tuple(reversed(x))] for b in range(N)]
            h0, h1 = h_funcs(ph0), h_funcs(ph1)
            mu = [self.at(st["mu"], i, x) for i in range(nc)]
            T0, T1 = self.temperature(x, n), self.temperature(x, n + 1)
            Delta = (-dt * divJ[x] - sum(self.C(b, mu, T0) * (h1[b] - h0[b]) for b in range(N))
                     - sum(h1[b] * (self.C(b, mu, T1) - self.C(b, mu, T0)) for b in range(N)))
            chit = sum(h1) * chi
            m = np.array(mu) + np.linalg.solve(chit, Delta)
            for i in range(nc):
                new[(i,) + tuple(reversed(x))] = m[i]
        return new

    # ----- lattice Boltzmann -----
    def lbm(self, st, phin, mun):
        cf, d, Q, N = self.cfg, self.dim, self.Q, self.N
        tau = cf["tau_lb"]
        fpost = np.zeros_like(st["f"])
        unew = np.zeros_like(st["u"])
        for x in self.cells():
            f = [self.at(st["f"], k, x) for k in range(Q)]
            rho = sum(f)
            m = [sum(f[k] * self.c[k][a] for k in range(Q)) for a in range(d)]
            phil = phin[(N - 1,) + tuple(reversed(x))]
            mu = [mun[(i,) + tuple(reversed(x))] for i in range(self.nc)]
            Cl = self.C(N - 1, mu, self.temperature(x, st["step"] + 1))
            b = sum(cf["gbeta"][i] * (Cl[i] - cf["c_ref"][i]) for i in range(self.nc))
            FB = [0.0] * d
            FB[cf["grav_axis"]] = -rho * phil * b * cf["grav_sign"]
            # shrinkage: eta_b times the change of phi_b over the step along the
            # unit normal of phi^{n+1}_b (central differences)
            for bb, eta in enumerate(cf.get("eta", [0.0] * 3)[:N]):
                if eta == 0.0:
                    continue
                g = [self.gradc(dict(phi=phin), bb, x, e) for e in range(d)]
                gg = sum(v * v for v in g)
                if gg > 1e-24:
                    dphi = phin[(bb,) + tuple(reversed(x))] - st["phi"][(bb,) + tuple(reversed(x))]
                    for a in range(d):
                        FB[a] += eta * dphi * g[a] / gg ** 0.5
            nu = (tau - 0.5) / 3
            kap = 2 * nu * cf["h_drag"] / cf["W0"] * (1 - phil) ** 2
            if phil == 0:
                u = [0.0] * d
            else:
                u = [(m[a] + 0.5 * FB[a]) / (rho * (1 + 0.5 * kap)) for a in range(d)]
            F = [FB[a] - kap * rho * u[a] for a in range(d)]
            uu = sum(v * v for v in u)
            for k in range(Q):
                ck = self.c[k][:d]
                cu = sum(ck[a] * u[a] for a in range(d))
                feq = self.w[k] * rho * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * uu)
                S = (1 - 0.5 / tau) * self.w[k] * sum((3 * (ck[a] - u[a]) + 9 * cu * ck[a]) * F[a]
                                                      for a in range(d))
                fpost[(k,) + tuple(reversed(x))] = f[k] - (f[k] - feq) / tau + S
            for a in range(d):
                unew[(a,) + tuple(reversed(x))] = u[a]
        fnew = np.zeros_like(fpost)
        opp = [self.c.index(tuple(-v for v in ck)) for ck in self.c]
        for x in self.cells():
            for k in range(Q):
                src = self.inside(tuple(x[a] - self.c[k][a] for a in range(d)))
                if src is not None:
                    val = fpost[(k,) + tuple(reversed(src))]
                else:
                    val = fpost[(opp[k],) + tuple(reversed(x))]
                    if not self.per[1] and x[1] - self.c[k][1] >= self.n[1]:
                        val += 6 * self.w[k] * cf["rho0"] * self.c[k][0] * cf.get("lid_u", 0.0)
                fnew[(k,) + tuple(reversed(x))] = val
        return fnew, unew

    def step(self, st):
        phin = self.pf(st)
        mun = self.mu_update(st, phin)
        fnew, unew = self.lbm(st, phin, mun)
        return dict(phi=phin, mu=mun, f=fnew, u=unew, step=st["step"] + 1)
