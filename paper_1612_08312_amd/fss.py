"""Finite-size-scaling production driver (Sec. 2 protocol, Sec. 3 analysis).

The paper's measurement protocol (Sec. 2): for every lattice size L and
temperature T, discard the first sweeps of a run, measure the following
ones, and repeat with several independent runs; averages are taken over the
runs and the errors come from their spread.  Its analysis (Sec. 3.1-3.3):

  * the moment ratio U(T) = <m^4> / <m^2>^2 with m = M/N (Eq. 2) of
    different sizes crosses near T_c;
  * U collapses onto one curve as a function of t (N^(1/3))^(1/nu), with
    t = (T - T_c)/T_c and N^(1/3) = 16^(1/3) L as the linear size (Eq. 3);
  * <m^2> (N^(1/3))^(2 beta/nu) collapses against the same variable (Eq. 4).

All sweeps run on the GPU through one `Group` per model (every member's
trajectory is that of the lattice swept alone).  The host only reduces the
per-sweep records of the device into moments, errors and fits.

Readings where the paper leaves the choice open:
  * a run's estimate of <m^k> is the mean over its measured sweeps; the
    estimate over R runs is the mean of the R run means, and U is formed
    from the averaged moments (the ratio of means, not the mean of ratios);
  * errors are the jackknife over runs (leave one run out, R - 1 scaling);
    for a plain mean this equals the standard error of the run means;
  * the crossing of two sizes is a root of a weighted least-squares cubic
    through U_L1(T) - U_L2(T) over the scanned temperatures;
  * the collapse is scored by the quality measure of Houdayer and Hartmann
    (Phys. Rev. B 70, 014418 (2004)): each point is compared with the
    interpolation of every other size at the same scaling variable, in
    units of the combined error, and the mean of the squared deviations is
    minimised over the scaling parameters; the interpolation is quadratic
    (three nearest points) rather than their linear one, whose curvature
    bias pulled beta/nu low on synthetic data.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time
from dataclasses import dataclass, field

import numpy as np

from . import workloads

SIZE_FACTOR = 16.0 ** (1.0 / 3.0)  # N^(1/3) = 16^(1/3) L (Sec. 3.1)


def linear_size(L, lattice="pyro"):
    """The linear size used in the scaling variable: N^(1/3), with N = 16 L^3
    for the pyrochlore and N = L^3 for the simple-cubic lattice (Sec. 3.4)."""
    f = SIZE_FACTOR if lattice == "pyro" else 1.0
    return f * np.asarray(L, dtype=np.float64)


# ---------------------------------------------------------------------------
# Protocol and GPU runs


@dataclass
class Protocol:
    """What one finite-size-scaling scan runs: every (L, T, run) is one
    lattice with its own seed and a random start (Sec. 2: 10^4 discarded and
    2 x 10^5 measured sweeps, five runs, L = 32, 48, 64, 96)."""

    model: int
    Ls: tuple
    temps: tuple
    discard: int = 10_000
    measure: int = 200_000
    runs: int = 5
    seed: int = 1
    J: float = 1.0
    chunk: int = 1000  # sweeps per group call (records drained in between)
    autotune: bool = True
    lattice: str = "pyro"  # or "sc": the simple-cubic lattice on the generic graph path

    def members(self):
        """(L, T index, run, seed) of every lattice, in a fixed order; seeds
        are seed + position, so every lattice draws its own stream."""
        out = []
        for li, L in enumerate(self.Ls):
            for ti in range(len(self.temps)):
                for r in range(self.runs):
                    k = (li * len(self.temps) + ti) * self.runs + r
                    out.append((int(L), ti, r, self.seed + k))
        return out

    def sweeps_per_member(self):
        return self.discard + self.measure


# Half-width of the default window, relative to T_c: the scaling variable
# t (N^(1/3))^(1/nu) then spans about +-0.6 to +-1 at L = 32 for every model
# (U of the continuous models varies more slowly with it).
WINDOW = {workloads.ISING: 6e-4, workloads.XY: 1.2e-3, workloads.HEISENBERG: 2e-3}


def default_temperatures(model: int, n: int = 13, rel_halfwidth: float = None):
    """n temperatures spaced evenly over T_c (1 +- rel_halfwidth) around the
    paper's estimate of T_c (the window only sets where to look)."""
    tc = workloads.TC[model]
    rel_halfwidth = WINDOW[model] if rel_halfwidth is None else rel_halfwidth
    return tuple(float(t) for t in tc * (1.0 + np.linspace(-rel_halfwidth, rel_halfwidth, n)))


@dataclass
class RunData:
    """Per-lattice measured series: m2[L][ti][r] and m4[L][ti][r] arrays."""

    protocol: Protocol
    m2: dict = field(default_factory=dict)
    m4: dict = field(default_factory=dict)
    seconds: float = 0.0
    spin_updates: float = 0.0


def run_protocol(p: Protocol, device: str = "cuda:0", log=None) -> RunData:
    """Run every lattice of the protocol on the GPU and collect m^2, m^4 of
    the measured sweeps.  ``log`` (callable) receives progress lines."""
    import torch

    from . import pyrosw

    log = log or (lambda s: None)
    members = p.members()
    if p.lattice == "pyro":
        lats = [pyrosw.Lattice(L=L, model=p.model, T=p.temps[ti], J=p.J, seed=s,
                               start=pyrosw.PYRO_START_RANDOM, device=device)
                for (L, ti, r, s) in members]
        g = pyrosw.Group(lats)
        if p.autotune:
            g.autotune(3)
        sweep_all = g.sweep
        sites = lambda L: 16 * L ** 3
    elif p.lattice == "sc":
        # one generic-graph handle per lattice, each on its own stream
        tables = {L: pyrosw.simple_cubic_bonds(L) for L in set(m[0] for m in members)}
        lats = [pyrosw.Graph(tables[L], L ** 3, p.model, p.temps[ti], J=p.J, seed=s,
                             start=pyrosw.PYRO_START_RANDOM, device=device, stream=0)
                for (L, ti, r, s) in members]
        g = None

        def sweep_all(n):
            for lt in lats:
                lt.sweep(n)

        sites = lambda L: L ** 3
    else:
        raise ValueError("lattice must be 'pyro' or 'sc'")
    data = RunData(protocol=p)
    series = [([], []) for _ in members]
    try:
        total = p.sweeps_per_member()
        torch.cuda.synchronize(device)
        t0 = time.perf_counter()
        done = 0
        while done < total:
            n = min(p.chunk, total - done)
            sweep_all(n)
            for k, lt in enumerate(lats):
                rec = lt.moments()
                keep = rec[rec["sweep"] >= p.discard]  # sweep indices start at 0
                if len(keep):
                    series[k][0].append(keep["m2"].copy())
                    series[k][1].append(keep["m4"].copy())
            done += n
            log("fss: model %d, %d of %d sweeps, %.1f s" % (p.model, done, total, time.perf_counter() - t0))
        torch.cuda.synchronize(device)
        data.seconds = time.perf_counter() - t0
    finally:
        if g is not None:
            g.close()
        for lt in lats:
            lt.close()
    data.spin_updates = float(sum(sites(L) for (L, _, _, _) in members)) * p.sweeps_per_member()
    for k, (L, ti, r, _) in enumerate(members):
        data.m2.setdefault(L, {}).setdefault(ti, {})[r] = np.concatenate(series[k][0])
        data.m4.setdefault(L, {}).setdefault(ti, {})[r] = np.concatenate(series[k][1])
    return data


# ---------------------------------------------------------------------------
# Estimates and errors


def jackknife(values: np.ndarray, fn):
    """Jackknife over the first axis of ``values`` (one row per run):
    returns fn(all rows) and the error sqrt((R-1)/R sum (fn_(i) - mean)^2)."""
    values = np.asarray(values)
    R = values.shape[0]
    full = np.asarray(fn(values), dtype=np.float64)
    if R < 2:
        return full, np.full_like(full, np.nan)
    loo = np.array([fn(np.delete(values, i, axis=0)) for i in range(R)], dtype=np.float64)
    err = np.sqrt((R - 1) / R * np.sum((loo - loo.mean(axis=0)) ** 2, axis=0))
    return full, err


def run_means(data: RunData):
    """Per-run means of m^2 and m^4: arrays [L index][T index][run][2]."""
    p = data.protocol
    out = np.zeros((len(p.Ls), len(p.temps), p.runs, 2))
    for li, L in enumerate(p.Ls):
        for ti in range(len(p.temps)):
            for r in range(p.runs):
                out[li, ti, r, 0] = np.mean(data.m2[int(L)][ti][r])
                out[li, ti, r, 1] = np.mean(data.m4[int(L)][ti][r])
    return out


def moments_from_runs(rm: np.ndarray):
    """U and <m^2> from per-run means rm[..., run, 2] (runs on axis -2)."""
    m2 = rm[..., 0].mean(axis=-1)
    m4 = rm[..., 1].mean(axis=-1)
    return m4 / m2 ** 2, m2


def estimates(rm: np.ndarray):
    """U, dU, <m^2>, d<m^2> per (L, T) from per-run means [L][T][run][2],
    errors by the jackknife over runs."""
    runs_first = np.moveaxis(rm, 2, 0)  # [run][L][T][2]

    def fn(v):
        return np.stack(moments_from_runs(np.moveaxis(v, 0, 2)))

    est, err = jackknife(runs_first, fn)
    return est[0], err[0], est[1], err[1]


# ---------------------------------------------------------------------------
# Binder crossings


def line_root(x, y, w=None):
    """Root of the weighted least-squares line through (x, y)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    w = np.ones_like(x) if w is None else np.asarray(w, dtype=np.float64)
    xm = np.sum(w * x) / np.sum(w)
    ym = np.sum(w * y) / np.sum(w)
    slope = np.sum(w * (x - xm) * (y - ym)) / np.sum(w * (x - xm) ** 2)
    return xm - ym / slope


def crossing(temps, u1, u2, du1=None, du2=None, degree=3):
    """Temperature where U of two sizes cross: the root, nearest the root of
    a weighted straight line, of a weighted least-squares polynomial (cubic
    by default, fewer terms when there are few temperatures) through
    u1(T) - u2(T); weights 1/(du1^2 + du2^2) when errors are given.  The
    cubic follows the odd bend of the difference of two sigmoid curves
    about their crossing, which a straight line over a wide window does not."""
    T = np.asarray(temps, dtype=np.float64)
    d = np.asarray(u1, dtype=np.float64) - np.asarray(u2, dtype=np.float64)
    w = None
    if du1 is not None and du2 is not None:
        var = np.asarray(du1) ** 2 + np.asarray(du2) ** 2
        if np.all(var > 0):
            w = 1.0 / var
    x0 = float(line_root(T, d, w))
    deg = max(1, min(degree, len(T) - 2))
    if deg == 1:
        return x0
    mid, half = 0.5 * (T[0] + T[-1]), 0.5 * abs(T[-1] - T[0])
    z = (T - mid) / half
    c = np.polyfit(z, d, deg, w=None if w is None else np.sqrt(w))
    r = np.roots(c)
    r = r[np.abs(r.imag) < 1e-12].real
    r = r[np.abs(r) <= 1.0] * half + mid
    if len(r) == 0:
        return x0
    return float(r[np.argmin(np.abs(r - x0))])


def crossings(temps, rm: np.ndarray, Ls):
    """Crossing temperature of every pair of successive sizes, with its
    jackknife error over runs: list of (L1, L2, T_x, dT_x)."""
    U, dU, _, _ = estimates(rm)
    out = []
    runs_first = np.moveaxis(rm, 2, 0)
    for a in range(len(Ls) - 1):
        def fn(v, a=a):
            u, _ = moments_from_runs(np.moveaxis(v, 0, 2))
            return crossing(temps, u[a], u[a + 1], dU[a], dU[a + 1])

        tx, err = jackknife(runs_first, fn)
        out.append((int(Ls[a]), int(Ls[a + 1]), float(tx), float(err)))
    return out


# ---------------------------------------------------------------------------
# Data collapse


# Interpolation order of the collapse measure: 2 (three-point Lagrange)
# unless a caller asks for Houdayer and Hartmann's linear interpolation (1).
COLLAPSE_ORDER = 2


def collapse_quality(xs, ys, dys, order=None):
    """Houdayer-Hartmann quality of a collapse: xs, ys, dys are lists (one
    entry per size) of arrays sorted by x.  For every point and every other
    size whose x range brackets it, the other size's value and error are
    interpolated at that x (order 1: linearly between the two bracketing
    points, as Houdayer and Hartmann do; order 2: through the three nearest
    points, which removes the curvature bias of the linear form on coarse
    grids); the result is the mean of (y - Y)^2 / (dy^2 + dY^2) over all such
    comparisons (inf if none)."""
    order = COLLAPSE_ORDER if order is None else order
    total, count = 0.0, 0
    for i in range(len(xs)):
        for j in range(len(xs)):
            if i == j:
                continue
            xj, yj, dyj = xs[j], ys[j], dys[j]
            n = len(xj)
            for x, y, dy in zip(xs[i], ys[i], dys[i]):
                if x < xj[0] or x > xj[-1]:
                    continue
                if order == 2 and n >= 3:
                    m = int(np.argmin(np.abs(xj - x)))
                    m = min(max(m, 1), n - 2)
                    p = xj[m - 1:m + 2]
                    if p[0] == p[1] or p[1] == p[2]:
                        continue
                    w = np.array([(x - p[1]) * (x - p[2]) / ((p[0] - p[1]) * (p[0] - p[2])),
                                  (x - p[0]) * (x - p[2]) / ((p[1] - p[0]) * (p[1] - p[2])),
                                  (x - p[0]) * (x - p[1]) / ((p[2] - p[0]) * (p[2] - p[1]))])
                    Y = float(w @ yj[m - 1:m + 2])
                    dY2 = float((w * w) @ (dyj[m - 1:m + 2] ** 2))
                else:
                    k = int(np.searchsorted(xj, x, side="right")) - 1
                    k = min(max(k, 0), n - 2)
                    h = xj[k + 1] - xj[k]
                    f = 0.0 if h == 0 else (x - xj[k]) / h
                    Y = (1 - f) * yj[k] + f * yj[k + 1]
                    dY2 = ((1 - f) * dyj[k]) ** 2 + (f * dyj[k + 1]) ** 2
                total += (y - Y) ** 2 / (dy ** 2 + dY2)
                count += 1
    return total / count if count else math.inf


def _scaled(temps, Ls, tc, nu, values, errs, power=0.0, lattice="pyro", d1=1.0, d2=1.0):
    """Scaling variable D1 t Lp^(1/nu) and values Lp^power / D2 per size
    (sorted by the variable); D1 = D2 = 1 unless two lattices are compared
    (Sec. 3.4)."""
    xs, ys, dys = [], [], []
    T = np.asarray(temps, dtype=np.float64)
    for li, L in enumerate(Ls):
        lp = float(linear_size(L, lattice))
        x = d1 * (T - tc) / tc * lp ** (1.0 / nu)
        o = np.argsort(x)
        xs.append(x[o])
        ys.append(values[li][o] * lp ** power / d2)
        dys.append(errs[li][o] * lp ** power / d2)
    return xs, ys, dys


def fit_tc_nu(temps, Ls, U, dU, tc0, nu0, lattice="pyro", order=None):
    """T_c and nu minimising the collapse quality of U (Eq. 3)."""
    from scipy.optimize import minimize

    def cost(v):
        tc, nu = v
        if nu <= 0.05:
            return 1e30
        return collapse_quality(*_scaled(temps, Ls, tc, nu, U, dU, lattice=lattice), order=order)

    best = minimize(cost, x0=[tc0, nu0], method="Nelder-Mead",
                    options=dict(xatol=1e-7, fatol=1e-9, maxiter=4000,
                                 initial_simplex=[[tc0, nu0], [tc0 * (1 + 2e-4), nu0], [tc0, nu0 * 1.1]]))
    return float(best.x[0]), float(best.x[1]), float(best.fun)


def fit_beta_nu(temps, Ls, m2, dm2, tc, nu, lo=0.2, hi=0.9, lattice="pyro", order=None):
    """beta/nu minimising the collapse quality of <m^2> (N^(1/3))^(2 beta/nu)
    at fixed T_c and nu (Eq. 4)."""
    from scipy.optimize import minimize_scalar

    def cost(bn):
        return collapse_quality(*_scaled(temps, Ls, tc, nu, m2, dm2, power=2.0 * bn, lattice=lattice), order=order)

    best = minimize_scalar(cost, bounds=(lo, hi), method="bounded", options=dict(xatol=1e-6))
    return float(best.x), float(best.fun)


def collapse_fit(temps, Ls, rm: np.ndarray, tc0: float, nu0: float, lattice="pyro", order=None):
    """T_c, nu and beta/nu from the collapses of U and <m^2> with the given
    interpolation order of the collapse measure, errors by the jackknife over
    runs (the fits redone with one run left out)."""
    U, dU, m2, dm2 = estimates(rm)
    tc, nu, q = fit_tc_nu(temps, Ls, U, dU, tc0, nu0, lattice, order)
    bn, qb = fit_beta_nu(temps, Ls, m2, dm2, tc, nu, lattice=lattice, order=order)
    runs_first = np.moveaxis(rm, 2, 0)

    def refit(v):
        sub = np.moveaxis(v, 0, 2)
        u, du, mm, dmm = estimates(sub)
        t, n, _ = fit_tc_nu(temps, Ls, u, du, tc, nu, lattice, order)
        b, _ = fit_beta_nu(temps, Ls, mm, dmm, t, n, lattice=lattice, order=order)
        return np.array([t, n, b])

    R = rm.shape[2]
    if R >= 3:
        loo = np.array([refit(np.delete(runs_first, i, axis=0)) for i in range(R)])
        err = np.sqrt((R - 1) / R * np.sum((loo - loo.mean(axis=0)) ** 2, axis=0))
    else:
        err = np.full(3, np.nan)
    return dict(Tc=tc, dTc=float(err[0]), nu=nu, dnu=float(err[1]), beta_over_nu=bn, dbeta_over_nu=float(err[2]),
                quality_U=q, quality_m2=qb)


def analyse(temps, Ls, rm: np.ndarray, tc0: float, nu0: float, lattice="pyro"):
    """Everything the paper extracts from one model's scan: U and <m^2>
    tables, Binder crossings, T_c, nu, beta/nu (jackknife errors).  The
    collapse fits are reported with the default three-point measure and,
    side by side, with Houdayer and Hartmann's linear one (collapse_linear)."""
    U, dU, m2, dm2 = estimates(rm)
    res = dict(U=U.tolist(), dU=dU.tolist(), m2=m2.tolist(), dm2=dm2.tolist(),
               crossings=[dict(L1=a, L2=b, T=t, dT=e) for (a, b, t, e) in crossings(temps, rm, Ls)])
    res.update(collapse_fit(temps, Ls, rm, tc0, nu0, lattice, order=COLLAPSE_ORDER))
    res["collapse_order"] = COLLAPSE_ORDER
    res["collapse_linear"] = collapse_fit(temps, Ls, rm, tc0, nu0, lattice, order=1)
    return res


def universal_factors(pyro: dict, sc: dict, nu: float, bn: float):
    """Nonuniversal metric factors of the pyrochlore lattice against the
    simple cubic (Sec. 3.4): with D1 = D2 = 1 for the simple cubic, D1
    minimises the collapse quality of U against D1 t (N^(1/3))^(1/nu) over
    the sizes of both lattices, then D2 that of <m^2> (N^(1/3))^(2 beta/nu) / D2
    at that D1.  Each lattice uses its own T_c.  ``pyro`` and ``sc`` hold
    temps, L, Tc and run_means as written by a scan; errors are the
    jackknife over runs (run r of both lattices left out together)."""
    from scipy.optimize import minimize_scalar

    rp, rs = np.asarray(pyro["run_means"]), np.asarray(sc["run_means"])

    def fit(rp, rs):
        Up, dUp, mp, dmp = estimates(rp)
        Us, dUs, ms, dms = estimates(rs)
        sc_u = _scaled(sc["temps"], sc["L"], sc["Tc"], nu, Us, dUs, lattice="sc")
        sc_m = _scaled(sc["temps"], sc["L"], sc["Tc"], nu, ms, dms, power=2.0 * bn, lattice="sc")

        def cost1(d1):
            cp = _scaled(pyro["temps"], pyro["L"], pyro["Tc"], nu, Up, dUp, d1=d1)
            return collapse_quality(*[a + b for a, b in zip(cp, sc_u)])

        d1 = minimize_scalar(cost1, bounds=(0.3, 3.0), method="bounded", options=dict(xatol=1e-6)).x

        def cost2(d2):
            cp = _scaled(pyro["temps"], pyro["L"], pyro["Tc"], nu, mp, dmp, power=2.0 * bn, d1=d1, d2=d2)
            return collapse_quality(*[a + b for a, b in zip(cp, sc_m)])

        d2 = minimize_scalar(cost2, bounds=(0.3, 3.0), method="bounded", options=dict(xatol=1e-6)).x
        return np.array([d1, d2, cost1(d1), cost2(d2)])

    full = fit(rp, rs)
    R = min(rp.shape[2], rs.shape[2])
    err = np.full(2, np.nan)
    if R >= 3:
        loo = np.array([fit(np.delete(rp, i, axis=2), np.delete(rs, i, axis=2))[:2] for i in range(R)])
        err = np.sqrt((R - 1) / R * np.sum((loo - loo.mean(axis=0)) ** 2, axis=0))
    return dict(D1=float(full[0]), dD1=float(err[0]), D2=float(full[1]), dD2=float(err[1]),
                quality_U=float(full[2]), quality_m2=float(full[3]))


# Simple-cubic critical temperatures the paper quotes from the literature
# (Sec. 3.1-3.3) and its metric factors of the pyrochlore lattice (Sec. 3.4).
SC_TC = {workloads.ISING: 4.511524, workloads.XY: 2.20182, workloads.HEISENBERG: 1.4430}
PAPER_D = {workloads.ISING: (1.0, 0.91), workloads.XY: (0.96, 0.91), workloads.HEISENBERG: (0.92, 0.91)}

# Estimates the paper prints (Sec. 3.1-3.3): T_c, nu, beta/nu with the error
# in the last digits.
PAPER = {
    workloads.ISING: dict(Tc=(4.21394, 2e-5), nu=(0.629, 0.002), beta_over_nu=(0.520, 0.005)),
    workloads.XY: dict(Tc=(2.02850, 2e-5), nu=(0.672, 0.002), beta_over_nu=(0.515, 0.005)),
    workloads.HEISENBERG: dict(Tc=(1.31695, 2e-5), nu=(0.711, 0.002), beta_over_nu=(0.515, 0.005)),
}


def main(argv=None):
    ap = argparse.ArgumentParser(description="Finite-size-scaling scan of one model on the GPU")
    ap.add_argument("--model", type=int, default=1, choices=(1, 2, 3))
    ap.add_argument("--lattice", default="pyro", choices=("pyro", "sc"))
    ap.add_argument("--universal", nargs=2, metavar=("PYRO_JSON", "SC_JSON"), default=None,
                    help="no scan: metric factors D1, D2 from two scans' output (Sec. 3.4)")
    ap.add_argument("--L", type=int, nargs="+", default=[32, 48, 64, 96])
    ap.add_argument("--temps", type=float, nargs="*", default=None,
                    help="temperatures (default: 13 over T_c (1 +- w), w from WINDOW)")
    ap.add_argument("--discard", type=int, default=10_000)
    ap.add_argument("--measure", type=int, default=200_000)
    ap.add_argument("--runs", type=int, default=5)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--chunk", type=int, default=1000)
    args = ap.parse_args(argv)
    if args.universal:
        pyro, sc = (json.loads(open(f).read().strip().splitlines()[-1]) for f in args.universal)
        ref = PAPER[pyro["model"]]
        res = universal_factors(pyro, sc, ref["nu"][0], ref["beta_over_nu"][0])
        res.update(model=pyro["model"], paper_D1_D2=PAPER_D[pyro["model"]])
        print(json.dumps(res))
        return
    tc_ref = PAPER[args.model]["Tc"][0] if args.lattice == "pyro" else SC_TC[args.model]
    temps = tuple(args.temps) if args.temps else tuple(
        float(t) for t in tc_ref * (1.0 + np.linspace(-WINDOW[args.model], WINDOW[args.model], 13)))
    p = Protocol(model=args.model, Ls=tuple(args.L), temps=temps, discard=args.discard,
                 measure=args.measure, runs=args.runs, seed=args.seed, chunk=args.chunk, lattice=args.lattice)
    data = run_protocol(p, log=lambda s: print(s, file=sys.stderr, flush=True))
    ref = PAPER[args.model]
    rm = run_means(data)
    res = analyse(temps, p.Ls, rm, tc_ref, ref["nu"][0], args.lattice)
    res.update(model=args.model, lattice=args.lattice, L=list(p.Ls), temps=list(temps), discard=p.discard,
               measure=p.measure, runs=p.runs, seconds=data.seconds,
               spin_updates_per_s=data.spin_updates / data.seconds, paper=ref, run_means=rm.tolist())
    print(json.dumps(res))


if __name__ == "__main__":
    main()
