"""Independent reference solutions that pin the CPU oracle.

Nothing here calls the oracle or the GPU library.  These are the mathematics
the method must reproduce:

* closed forms of the transport problem (purely absorbing slabs under beam,
  uniform and cosine incidence; infinite-medium steady and pulsed fluxes,
  one-group and multigroup through a matrix exponential; the uncollided
  flux of an isotropic plane pulse);
* a discrete-ordinates (S_N) slab solver for a scattering slab;
* the 63-bit LCG in Python big integers, with its closed-form skip-ahead;
* a separately written pure-Python event-by-event tracer of the same
  algorithm for bit-level comparison on tiny inputs.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
from scipy import linalg, special
from scipy.signal import lfilter

# ---------------------------------------------------------------------------
# 63-bit LCG in big integers
# ---------------------------------------------------------------------------

LCG_G = 2806196910506780709
LCG_C = 1
LCG_STRIDE = 152917
MOD = 1 << 63


def lcg_skip_closed_form(s: int, k: int) -> int:
    """s_k = g^k s + c (g^k - 1) / (g - 1)  (mod 2^63).

    (g^k - 1)/(g - 1) mod 2^63 is computed exactly as
    (g^k mod (g - 1) 2^63 - 1) // (g - 1)."""
    gk_big = pow(LCG_G, k, (LCG_G - 1) * MOD)
    geom = (gk_big - 1) // (LCG_G - 1)
    return (pow(LCG_G, k, MOD) * s + LCG_C * geom) % MOD


def lcg_step(s: int) -> int:
    return (LCG_G * s + LCG_C) % MOD


def xi_of(s: int) -> float:
    return (s >> 10) / float(1 << 53)


# ---------------------------------------------------------------------------
# Closed forms (per source particle)
# ---------------------------------------------------------------------------

def En(n, x):
    return special.expn(n, x)


def slab_absorber_bins(edges, sigma_t, law):
    """Bin-averaged uncollided scalar flux in a purely absorbing half-space
    lit at x=0 by a unit current with the given angular law.

    beam:    phi(x) = exp(-St x)
    uniform: mu uniform on (0,1]   -> phi(x) = E1(St x)
    cosine:  incident flux isotropic -> phi(x) = 2 E2(St x)
    """
    a, b = edges[:-1], edges[1:]
    dx = b - a
    St = sigma_t
    if law == "beam":
        return (np.exp(-St * a) - np.exp(-St * b)) / (St * dx)
    if law == "uniform":
        return (En(2, St * a) - En(2, St * b)) / (St * dx)
    if law == "cosine":
        return 2.0 * (En(3, St * a) - En(3, St * b)) / (St * dx)
    raise ValueError(law)


def slab_absorber_transmission(L, sigma_t, law):
    tau = sigma_t * L
    return {"beam": math.exp(-tau), "uniform": float(En(2, tau)),
            "cosine": float(2.0 * En(3, tau))}[law]


def removal_matrix(sigma_t, sigma_s, fission=None):
    """M[g, g'] = Sigma_t,g delta_gg' - Sigma_s(g' -> g) for one material;
    sigma_s is indexed [from, to].  With fission = (sigma_f, nu, chi) the
    prompt production chi_g nu_g' Sigma_f,g' is subtracted as well."""
    M = np.diag(sigma_t) - np.asarray(sigma_s).T
    if fission is not None:
        sf, nu, chi = (np.asarray(a, dtype=float).ravel() for a in fission)
        M = M - np.outer(chi, nu * sf)
    return M


def infinite_medium_steady(sigma_t, sigma_s, volume, fission=None):
    """Scalar flux per group in an infinite medium with a uniform source of
    one particle in group 0 spread over the given volume: phi = M^-1 S."""
    G = len(sigma_t)
    S = np.zeros(G)
    S[0] = 1.0 / volume
    return np.linalg.solve(removal_matrix(sigma_t, sigma_s, fission), S)


def infinite_medium_pulse_bins(sigma_t, sigma_s, speed, edges, volume, fission=None):
    """Time-bin averages of phi(t) = V exp(-M V t) n0 with n0 = one particle
    in group 0 per volume:  V (M V)^-1 (e^{-MV ta} - e^{-MV tb}) n0 / dt.
    Returns [K, G]."""
    G = len(sigma_t)
    V = np.diag(speed)
    A = removal_matrix(sigma_t, sigma_s, fission) @ V
    n0 = np.zeros(G)
    n0[0] = 1.0 / volume
    out = []
    Ainv = np.linalg.inv(A)
    for ta, tb in zip(edges[:-1], edges[1:]):
        d = (linalg.expm(-A * ta) - linalg.expm(-A * tb)) @ n0
        out.append(V @ Ainv @ d / (tb - ta))
    return np.array(out)


def infinite_medium_pulse_points(sigma_t, sigma_s, speed, times, volume, fission=None):
    """Point values phi(t) = V exp(-M V t) n0 at the given times (n0 = one
    particle in group 0 per volume).  Returns [len(times), G]."""
    G = len(sigma_t)
    V = np.diag(speed)
    A = removal_matrix(sigma_t, sigma_s, fission) @ V
    n0 = np.zeros(G)
    n0[0] = 1.0 / volume
    return np.array([V @ (linalg.expm(-A * t) @ n0) for t in times])


def plane_pulse_uncollided_point(x0, sigma_t, v, xa, xb, t):
    """Average over [xa, xb] of the uncollided flux of an isotropic plane
    pulse at x0 at time t > 0: e^{-St v t} / (2 t) on |x - x0| < v t."""
    lo = max(xa, x0 - v * t)
    hi = min(xb, x0 + v * t)
    return math.exp(-sigma_t * v * t) * max(0.0, hi - lo) / (2.0 * t * (xb - xa))


def plane_pulse_moments(c, t):
    """Population m00 and second spatial moment m20 = int x^2 n dx of an
    isotropic plane pulse at x = 0 in an infinite one-group medium with
    isotropic re-emission c per collision (Sigma_t = v = 1).  Moments
    m_kl = int int x^k mu^l psi dx dmu of the transport equation obey
    m_kl' = k m_{k-1,l+1} - m_kl + c a_l m_k0 with a_l = 1/(l+1) for even
    l, 0 for odd l; the set (m00, m02, m11, m20) is closed:
      m00' = (c-1) m00, m02' = (c/3) m00 - m02, m11' = m02 - m11,
      m20' = 2 m11 + (c-1) m20, starting from (1, 1/3, 0, 0)."""
    A = np.array([[c - 1.0, 0.0, 0.0, 0.0],
                  [c / 3.0, -1.0, 0.0, 0.0],
                  [0.0, 1.0, -1.0, 0.0],
                  [0.0, 0.0, 2.0, c - 1.0]])
    m = linalg.expm(A * t) @ np.array([1.0, 1.0 / 3.0, 0.0, 0.0])
    return m[0], m[3]


def pulse_population(c, t):
    """Particle population of an infinite one-group medium after a unit
    pulse, time in mean free times: exp((c - 1) t)."""
    return math.exp((c - 1.0) * t)


def plane_pulse_uncollided_bin(x0, sigma_t, v, xa, xb, ta, tb):
    """Space-time integral over [xa,xb] x [ta,tb] of the uncollided flux of
    an isotropic plane pulse at x0: phi_u = e^{-St v t} / (2 t) on
    |x - x0| < v t."""
    from scipy.integrate import quad

    def inner(t):
        lo = max(xa, x0 - v * t)
        hi = min(xb, x0 + v * t)
        w = max(0.0, hi - lo)
        return math.exp(-sigma_t * v * t) * w / (2.0 * t)

    brk = [t for t in (abs(xa - x0) / v, abs(xb - x0) / v) if ta < t < tb]
    val, _ = quad(inner, ta, tb, points=brk or None, limit=200, epsabs=1e-13, epsrel=1e-11)
    return val


# ---------------------------------------------------------------------------
# Discrete ordinates slab solver
# ---------------------------------------------------------------------------

def sn_slab(L, sigma_t, sigma_s, n_cells=4000, n_mu=64, tol=1e-12, law="cosine"):
    """One-group slab [0, L], vacuum on both faces, isotropic scattering,
    lit at x = 0 by a unit current with the given law.  Uncollided flux is
    analytic; the collided flux solves mu dpsi/dx + St psi = (Ss/2) phi with
    diamond differencing and source iteration.  Returns (cell edges, cell
    average scalar flux) on the fine mesh, and a function mapping coarse
    bin edges to bin averages (uncollided part exact)."""
    h = L / n_cells
    xe = np.linspace(0.0, L, n_cells + 1)
    mu, wt = np.polynomial.legendre.leggauss(n_mu)
    # uncollided cell averages
    if law == "cosine":
        phi_u = 2.0 * (En(3, sigma_t * xe[:-1]) - En(3, sigma_t * xe[1:])) / (sigma_t * h)
    elif law == "uniform":
        phi_u = (En(2, sigma_t * xe[:-1]) - En(2, sigma_t * xe[1:])) / (sigma_t * h)
    else:
        phi_u = (np.exp(-sigma_t * xe[:-1]) - np.exp(-sigma_t * xe[1:])) / (sigma_t * h)
    phi_c = np.zeros(n_cells)
    for _ in range(2000):
        q = 0.5 * sigma_s * (phi_u + phi_c)
        new = np.zeros(n_cells)
        for m, w in zip(mu, wt):
            am = abs(m)
            a = (am / h - sigma_t / 2.0) / (am / h + sigma_t / 2.0)
            b = 1.0 / (am / h + sigma_t / 2.0)
            src = q if m > 0 else q[::-1]
            edge_out = lfilter([b], [1.0, -a], src)     # psi at outgoing edges, zero inflow
            edge_in = np.concatenate([[0.0], edge_out[:-1]])
            avg = 0.5 * (edge_in + edge_out)
            new += w * (avg if m > 0 else avg[::-1])
        diff = np.max(np.abs(new - phi_c))
        phi_c = new
        if diff < tol:
            break
    phi = phi_u + phi_c

    def bins(edges):
        out = []
        for a_, b_ in zip(edges[:-1], edges[1:]):
            i0 = int(round(a_ / h))
            i1 = int(round(b_ / h))
            out.append(phi_c[i0:i1].mean())
        coll = np.array(out)
        unc = slab_absorber_bins(np.asarray(edges), sigma_t, law)
        return unc + coll

    return xe, phi, bins


def _sn_sweep(q, sigma_t, h, mu, wt):
    """Scalar flux of mu dpsi/dx + St psi = q (isotropic q per unit mu,
    cell averages) on a uniform mesh with zero inflow at both faces, by
    diamond differencing in every direction of the quadrature."""
    out = np.zeros(q.size)
    for m, w in zip(mu, wt):
        am = abs(m)
        a = (am / h - sigma_t / 2.0) / (am / h + sigma_t / 2.0)
        b = 1.0 / (am / h + sigma_t / 2.0)
        src = q if m > 0 else q[::-1]
        edge_out = lfilter([b], [1.0, -a], src)
        edge_in = np.concatenate([[0.0], edge_out[:-1]])
        avg = 0.5 * (edge_in + edge_out)
        out += w * (avg if m > 0 else avg[::-1])
    return out


def sn_slab_mg(L, sigma_t, sigma_s, pmf, n_cells=2400, n_mu=64, tol=1e-12, law="cosine"):
    """G-group slab [0, L], vacuum on both faces, isotropic scattering with
    the transfer matrix sigma_s[g, g'] (from group g to g'), lit at x = 0 by
    a unit current whose group is g with probability pmf[g], entering with
    the given angular law.  The uncollided flux of each group is analytic;
    the collided flux of group g' solves
    mu dpsi/dx + St_g' psi = (1/2) sum_g Ss[g, g'] phi_g
    by diamond differencing, the groups swept in order and the sweeps
    repeated until the scattering source settles (up-scatter included).
    Returns a function mapping coarse bin edges to [G, bins] averages."""
    sigma_t = np.asarray(sigma_t, dtype=np.float64)
    sigma_s = np.asarray(sigma_s, dtype=np.float64)
    G = sigma_t.size
    h = L / n_cells
    xe = np.linspace(0.0, L, n_cells + 1)
    mu, wt = np.polynomial.legendre.leggauss(n_mu)
    phi_u = np.zeros((G, n_cells))
    for g in range(G):
        st = sigma_t[g]
        if law == "cosine":
            cell = 2.0 * (En(3, st * xe[:-1]) - En(3, st * xe[1:])) / (st * h)
        elif law == "uniform":
            cell = (En(2, st * xe[:-1]) - En(2, st * xe[1:])) / (st * h)
        else:
            cell = (np.exp(-st * xe[:-1]) - np.exp(-st * xe[1:])) / (st * h)
        phi_u[g] = pmf[g] * cell
    phi_c = np.zeros((G, n_cells))
    for _ in range(5000):
        diff = 0.0
        for g2 in range(G):
            q = 0.5 * sum(sigma_s[g, g2] * (phi_u[g] + phi_c[g]) for g in range(G))
            new = _sn_sweep(q, sigma_t[g2], h, mu, wt)
            diff = max(diff, float(np.max(np.abs(new - phi_c[g2]))))
            phi_c[g2] = new
        if diff < tol:
            break

    def bins(edges):
        edges = np.asarray(edges, dtype=np.float64)
        out = np.zeros((G, edges.size - 1))
        for j, (a_, b_) in enumerate(zip(edges[:-1], edges[1:])):
            i0, i1 = int(round(a_ / h)), int(round(b_ / h))
            out[:, j] = phi_c[:, i0:i1].mean(axis=1)
        for g in range(G):
            out[g] += pmf[g] * slab_absorber_bins(edges, sigma_t[g], law)
        return out

    return bins


def sn_slab_mg_volume(L, sigma_t, sigma_s, pmf, n_cells=2400, n_mu=64, tol=1e-12):
    """G-group slab [0, L], vacuum on both faces, with a unit isotropic
    source spread uniformly over the slab (group g with probability pmf[g])
    and isotropic scattering with the transfer matrix sigma_s[g, g'] (from
    g to g'): mu dpsi/dx + St_g' psi = (1/2)(pmf[g'] / L + sum_g
    Ss[g, g'] phi_g), swept as in sn_slab_mg.  Returns a function mapping
    coarse bin edges to [G, bins] averages of the scalar flux (track length
    per unit length per source particle)."""
    sigma_t = np.asarray(sigma_t, dtype=np.float64)
    sigma_s = np.asarray(sigma_s, dtype=np.float64)
    G = sigma_t.size
    h = L / n_cells
    mu, wt = np.polynomial.legendre.leggauss(n_mu)
    phi = np.zeros((G, n_cells))
    for _ in range(5000):
        diff = 0.0
        for g2 in range(G):
            q = 0.5 * (pmf[g2] / L + sum(sigma_s[g, g2] * phi[g] for g in range(G)))
            new = _sn_sweep(q, sigma_t[g2], h, mu, wt)
            diff = max(diff, float(np.max(np.abs(new - phi[g2]))))
            phi[g2] = new
        if diff < tol:
            break

    def bins(edges):
        edges = np.asarray(edges, dtype=np.float64)
        out = np.zeros((G, edges.size - 1))
        for j, (a_, b_) in enumerate(zip(edges[:-1], edges[1:])):
            i0, i1 = int(round(a_ / h)), int(round(b_ / h))
            out[:, j] = phi[:, i0:i1].mean(axis=1)
        return out

    return bins


def sn_slab_k(L, sigma_t, sigma_s, nu_sigma_f, n_cells=2000, n_mu=64, tol=1e-11):
    """One-group bare slab [0, L] (vacuum faces), isotropic scattering and
    fission: k-eigenvalue by power iteration on the fission source, each
    transport solve by source iteration with diamond differencing and
    Gauss-Legendre angles.  Returns (k, cell edges, cell-average flux per
    unit fission source: the fission source nu Sigma_f phi / k integrates
    to 1)."""
    h = L / n_cells
    xe = np.linspace(0.0, L, n_cells + 1)
    mu, wt = np.polynomial.legendre.leggauss(n_mu)

    def sweep(q):
        out = np.zeros(n_cells)
        for m, w in zip(mu, wt):
            am = abs(m)
            a = (am / h - sigma_t / 2.0) / (am / h + sigma_t / 2.0)
            b = 1.0 / (am / h + sigma_t / 2.0)
            src = q if m > 0 else q[::-1]
            edge_out = lfilter([b], [1.0, -a], src)
            edge_in = np.concatenate([[0.0], edge_out[:-1]])
            avg = 0.5 * (edge_in + edge_out)
            out += w * (avg if m > 0 else avg[::-1])
        return out

    phi = np.ones(n_cells)
    k = 1.0
    for _ in range(500):
        fis = nu_sigma_f * phi / k
        new = phi.copy()
        for _ in range(5000):
            nxt = sweep(0.5 * (sigma_s * new + fis))
            d = np.max(np.abs(nxt - new)) / np.max(np.abs(nxt))
            new = nxt
            if d < tol:
                break
        k_new = k * (nu_sigma_f * new).sum() / (nu_sigma_f * phi).sum()
        phi = new
        if abs(k_new - k) < tol:
            k = k_new
            break
        k = k_new
    phi = phi / ((nu_sigma_f * phi / k).sum() * h)
    return k, xe, phi


# ---------------------------------------------------------------------------
# Pure-Python tracer (bit-level brute force on tiny inputs)
# ---------------------------------------------------------------------------

def _fma(a: float, b: float, c: float) -> float:
    """Correctly rounded a*b + c through exact rationals."""
    return float(Fraction(a) * Fraction(b) + Fraction(c))


class PyTracer:
    """The transport algorithm written a second time, event by event, in
    plain Python floats.  Same readings as the oracle; no shared code."""

    def __init__(self, prob, N, seed):
        self.p = prob
        self.N = N
        self.seed = seed % MOD
        self.K = len(prob["tally"]["time_edges"]) - 1
        self.U = []
        for a in range(3):
            pl = list(prob["planes"][a])
            if not pl:
                self.U.append([])
                continue
            pts = set(pl) | set(prob["tally"]["mesh"][a])
            self.U.append(sorted(pts))
        st = prob["sigma_t"]
        ss = prob["sigma_s"]
        self.M, self.G = st.shape

    def _rn(self):
        self.s = lcg_step(self.s)
        return xi_of(self.s)

    def _iso(self):
        while True:
            a = 2.0 * self._rn() - 1.0
            b = 2.0 * self._rn() - 1.0
            r = a * a + b * b
            if r < 1.0:
                q = math.sqrt(1.0 - r)
                return [1.0 - 2.0 * r, (2.0 * a) * q, (2.0 * b) * q]

    def _mat(self, ix):
        c = []
        for a in range(3):
            if not self.U[a]:
                c.append(0)
                continue
            left = self.U[a][ix[a]]
            pl = self.p["planes"][a]
            j = max(i for i in range(len(pl) - 1) if pl[i] <= left)
            c.append(j)
        mat = self.p["material"]
        return int(mat[c[2], c[1], c[0]])

    def history(self, i):
        p = self.p
        self.s = lcg_skip_closed_form(self.seed, i * LCG_STRIDE)
        src = p["source"]
        x = []
        for a in range(3):
            xi = self._rn()
            x.append(src["lo"][a] + xi * (src["hi"][a] - src["lo"][a]) if self.U[a] else 0.0)
        xt = self._rn()
        t = src["t_lo"] + xt * (src["t_hi"] - src["t_lo"])
        xg = self._rn()
        run, g = 0.0, None
        pmf = list(src["group_pmf"])
        last = max(j for j in range(self.G) if pmf[j] > 0)
        for j in range(self.G):
            run += pmf[j]
            c = 1.0 if j >= last else run
            if xg < c:
                g = j
                break
        if src["kind"] == "isotropic":
            u = self._iso()
        else:
            xm = self._rn()
            law = src["mu_law"]
            mu = 1.0 if law == "beam" else (1.0 - xm if law == "uniform" else math.sqrt(1.0 - xm))
            while True:
                a = 2.0 * self._rn() - 1.0
                b = 2.0 * self._rn() - 1.0
                r = a * a + b * b
                if 0.0 < r < 1.0:
                    break
            cph = (a * a - b * b) / r
            sph = ((2.0 * a) * b) / r
            sn = math.sqrt(1.0 - mu * mu)
            ax = src["axis"]
            u = [0.0, 0.0, 0.0]
            u[ax] = float(src["sign"]) * mu
            u[(ax + 1) % 3] = sn * cph
            u[(ax + 2) % 3] = sn * sph
        inv = [1.0 / c if c != 0.0 else math.copysign(math.inf, c) for c in u]
        tau = -math.log(1.0 - self._rn())
        ix = []
        for a in range(3):
            if not self.U[a]:
                ix.append(0)
                continue
            P = self.U[a]
            j = max([k for k in range(len(P)) if P[k] <= x[a]], default=-1)
            if j >= 0 and x[a] == P[j] and u[a] < 0.0:
                j -= 1
            ix.append(min(max(j, 0), len(P) - 2))
        T = list(p["tally"]["time_edges"])
        rows = []
        if t >= T[-1]:
            return [[12.0, 0.0, x[0], x[1], x[2], t, g, self.K, tau]]
        k = max(j for j in range(self.K) if T[j] <= t)
        st_tab, ss_tab, v = p["sigma_t"], p["sigma_s"], p["speed"]
        while True:
            m = self._mat(ix)
            St = float(st_tab[m, g])
            dc = math.inf if St == 0.0 else tau * (1.0 / St)
            da = [math.inf] * 3
            for a in range(3):
                if not self.U[a] or u[a] == 0.0:
                    continue
                P = self.U[a][ix[a] + 1] if u[a] > 0.0 else self.U[a][ix[a]]
                da[a] = max((P - x[a]) * inv[a], 0.0)
            ds = min(da)
            Tn = T[k + 1]
            dt = math.inf if Tn == math.inf else max((Tn - t) * float(v[g]), 0.0)
            if dt <= ds and dt <= dc:
                ev, d = 0, dt
            elif ds <= dc:
                ev, d = 1, ds
            else:
                ev, d = 2, dc
            if d == math.inf:
                rows.append([ev, d, x[0], x[1], x[2], t, g, k, tau])
                rows.append([13.0, 0.0, x[0], x[1], x[2], t, g, k, tau])
                return rows
            x = [_fma(d, u[a], x[a]) for a in range(3)]
            t = Tn if ev == 0 else t + d * (1.0 / float(v[g]))
            if ev != 2 and St != 0.0:
                tau = max(tau - d * St, 0.0)
            term = None
            if ev == 0:
                k += 1
                if k == self.K:
                    term = 2
            elif ev == 1:
                for a in range(3):
                    if term is not None:
                        break
                    if not self.U[a] or da[a] != d:
                        continue
                    P = self.U[a]
                    n_cells = len(P) - 1
                    if u[a] > 0.0:
                        x[a] = P[ix[a] + 1]
                        face = 2 * a + 1 if ix[a] == n_cells - 1 else None
                        if face is None:
                            ix[a] += 1
                    else:
                        x[a] = P[ix[a]]
                        face = 2 * a if ix[a] == 0 else None
                        if face is None:
                            ix[a] -= 1
                    if face is not None:
                        if int(p["bc"][face]) == 0:
                            term = 1
                        else:
                            u[a] = -u[a]
                            inv[a] = -inv[a]
            else:
                row = ss_tab[m, g]
                Ss = 0.0
                for val in row:
                    Ss += float(val)
                ps = Ss / St
                if not (self._rn() < ps):
                    term = 0
                else:
                    xg = self._rn()
                    run = 0.0
                    last = max(j for j in range(self.G) if row[j] > 0.0)
                    for j in range(self.G):
                        run += float(row[j])
                        c = 1.0 if j >= last else run / Ss
                        if xg < c:
                            g = j
                            break
                    u = self._iso()
                    inv = [1.0 / c if c != 0.0 else math.copysign(math.inf, c) for c in u]
                    tau = -math.log(1.0 - self._rn())
            rows.append([ev, d, x[0], x[1], x[2], t, g, k, tau])
            if term is not None:
                rows.append([10.0 + term, 0.0, x[0], x[1], x[2], t, g, k, tau])
                return rows
