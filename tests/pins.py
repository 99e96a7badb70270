"""Independent checks that pin the CPU oracle to the paper and to exact
mathematics (no GPU).  Each function returns ``(ok, info)`` so that tests can
also assert that a mistake planted in the oracle makes the check fail.

None of this code calls the oracle's arithmetic: it enumerates, integrates
or simulates the model of Eq. (1) by other means (exact sums over states,
closed forms, a Metropolis sampler) and compares with oracle output handed
in by the caller.
"""
from __future__ import annotations

import itertools

import numpy as np
from scipy import special, stats


def pyro_positions(L: int) -> np.ndarray:
    """Site positions (units a/4) of the 16-site-cell pyrochlore lattice,
    in the project's site numbering: index 16*cell + 4*f + mu, cell =
    (z*L + y)*L + x, position 4*(x,y,z) + F_f + B_mu (Sec. 2)."""
    F = np.array([[0, 0, 0], [0, 2, 2], [2, 0, 2], [2, 2, 0]])
    B = np.array([[0, 0, 0], [0, 1, 1], [1, 0, 1], [1, 1, 0]])
    out = []
    for z in range(L):
        for y in range(L):
            for x in range(L):
                for f in range(4):
                    for mu in range(4):
                        out.append(4 * np.array([x, y, z]) + F[f] + B[mu])
    return np.array(out)


def nn_pairs_brute_force(pos: np.ndarray, box: int) -> set:
    """All unordered pairs at minimum-image squared distance 2 (nearest
    neighbours of the pyrochlore lattice in units of a/4)."""
    d = pos[:, None, :] - pos[None, :, :]
    d = (d + box // 2) % box - box // 2
    d2 = (d * d).sum(-1)
    i, j = np.nonzero(np.triu(d2 == 2, 1))
    return set(zip(i.tolist(), j.tolist()))


def binned_mean(x: np.ndarray, nbins: int = 50):
    """Mean and error from ``nbins`` consecutive bins (handles
    autocorrelation shorter than a bin)."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x) // nbins * nbins
    b = x[:n].reshape(nbins, -1).mean(axis=1)
    return float(b.mean()), float(b.std(ddof=1) / np.sqrt(nbins))


def binned_binder(m2: np.ndarray, m4: np.ndarray, nbins: int = 50):
    """U = <m4>/<m2>^2 with a jackknife error over bins."""
    n = len(m2) // nbins * nbins
    b2 = m2[:n].reshape(nbins, -1).mean(1)
    b4 = m4[:n].reshape(nbins, -1).mean(1)
    U = b4.mean() / b2.mean() ** 2
    jk = np.array([(b4.sum() - b4[k]) / (nbins - 1) / ((b2.sum() - b2[k]) / (nbins - 1)) ** 2
                   for k in range(nbins)])
    err = np.sqrt((nbins - 1) * np.mean((jk - jk.mean()) ** 2))
    return float(U), float(err)


# --------------------------------------------------------------------------
# Exact enumeration of the Ising model on a small graph.
# --------------------------------------------------------------------------
def ising_exact(N: int, a: np.ndarray, b: np.ndarray, T: float, J: float = 1.0, norm: int = None):
    """<E>, <m^2>, <m^4> and U by summing over all 2^N states (Eq. 1, Eq. 2);
    m = M / norm (default N; a diluted lattice passes its full site count)."""
    states = ((np.arange(2 ** N)[:, None] >> np.arange(N)[None, :]) & 1).astype(np.int64)
    s = 1 - 2 * states
    B = (s[:, a] * s[:, b]).sum(axis=1)
    E = -J * B
    w = np.exp(-(E - E.min()) / T)
    Z = w.sum()
    m = s.sum(axis=1) / (N if norm is None else norm)
    e_mean = float((w * E).sum() / Z)
    m2 = float((w * m ** 2).sum() / Z)
    m4 = float((w * m ** 4).sum() / Z)
    return dict(E=e_mean, m2=m2, m4=m4, U=m4 / m2 ** 2)


def check_against_exact(rec: np.ndarray, exact: dict, nsig: float = 4.5, discard: int = 100):
    r = rec[discard:]
    info = {}
    ok = True
    for key, field in (("E", "E"), ("m2", "m2"), ("m4", "m4")):
        mu, err = binned_mean(r[field])
        z = abs(mu - exact[key]) / max(err, 1e-300)
        info[key] = (mu, err, exact[key], z)
        ok &= bool(z < nsig)
    return ok, info


# --------------------------------------------------------------------------
# Exact Swendsen-Wang one-step transition matrix on a small Ising graph.
# --------------------------------------------------------------------------
def _components(N, edges):
    parent = list(range(N))

    def find(x):
        while parent[x] != x:
            x = parent[x]
        return x

    for i, j in edges:
        ri, rj = find(i), find(j)
        if ri != rj:
            parent[max(ri, rj)] = min(ri, rj)
    return [find(i) for i in range(N)]


def sw_transition_matrix(N: int, a, b, T: float, J: float = 1.0) -> np.ndarray:
    """P[s, s'] of one SW update: each parallel bond is occupied with
    probability 1 - exp(-2 J / T), then every cluster is flipped with
    probability 1/2.  States are bit patterns (bit k set = spin k down)."""
    p = 1.0 - np.exp(-2.0 * J / T)
    nb = len(a)
    P = np.zeros((2 ** N, 2 ** N))
    for s in range(2 ** N):
        spin = [1 - 2 * ((s >> k) & 1) for k in range(N)]
        par = [spin[a[e]] == spin[b[e]] for e in range(nb)]
        for occ in itertools.product((0, 1), repeat=nb):
            if any(o and not pa for o, pa in zip(occ, par)):
                continue
            w = 1.0
            for o, pa in zip(occ, par):
                if pa:
                    w *= p if o else (1.0 - p)
            if w == 0.0:
                continue
            comp = _components(N, [(a[e], b[e]) for e in range(nb) if occ[e]])
            roots = sorted(set(comp))
            for flips in itertools.product((0, 1), repeat=len(roots)):
                fl = dict(zip(roots, flips))
                s2 = s
                for k in range(N):
                    if fl[comp[k]]:
                        s2 ^= 1 << k
                P[s, s2] += w / 2 ** len(roots)
    return P


def boltzmann(N: int, a, b, T: float, J: float = 1.0) -> np.ndarray:
    states = ((np.arange(2 ** N)[:, None] >> np.arange(N)[None, :]) & 1)
    s = 1 - 2 * states
    E = -J * (s[:, a] * s[:, b]).sum(axis=1)
    w = np.exp(-(E - E.min()) / T)
    return w / w.sum()


def chi2_row(counts: np.ndarray, probs: np.ndarray, alpha: float = 1e-4):
    """Chi-square goodness of fit of observed counts to a distribution.
    Categories with zero probability must have zero counts."""
    n = counts.sum()
    if np.any(counts[probs == 0] > 0):
        return False, dict(reason="impossible state observed")
    m = probs > 0
    exp = n * probs[m]
    chi2 = float(((counts[m] - exp) ** 2 / exp).sum())
    dof = int(m.sum()) - 1
    pval = float(stats.chi2.sf(chi2, dof))
    return pval > alpha, dict(chi2=chi2, dof=dof, p=pval)


# --------------------------------------------------------------------------
# Two spins and one bond: closed forms of <s1 . s2> for the O(n) model.
# --------------------------------------------------------------------------
def single_bond_correlation(n: int, K: float) -> float:
    """<s1.s2> for H = -J s1.s2 with K = J/T: Ising tanh K; XY I1(K)/I0(K);
    Heisenberg coth K - 1/K."""
    if n == 1:
        return float(np.tanh(K))
    if n == 2:
        return float(special.i1(K) / special.i0(K))
    return float(1.0 / np.tanh(K) - 1.0 / K)


# --------------------------------------------------------------------------
# Independent single-spin Metropolis sampler for the O(n) model on a small
# graph (many independent chains in parallel).
# --------------------------------------------------------------------------
def metropolis_on(N: int, a, b, n: int, T: float, J: float = 1.0, chains: int = 2000,
                  sweeps: int = 3000, discard: int = 300, seed: int = 0):
    rng = np.random.default_rng(seed)
    nbrs = [[] for _ in range(N)]
    for x, y in zip(a, b):
        nbrs[x].append(y)
        nbrs[y].append(x)

    def rand_unit(size):
        v = rng.standard_normal((size, n))
        return v / np.linalg.norm(v, axis=1, keepdims=True)

    s = np.stack([rand_unit(chains) for _ in range(N)], axis=1)  # [chains, N, n]
    E_samples, m2_samples = [], []
    for sw in range(sweeps):
        for i in range(N):
            h = s[:, nbrs[i], :].sum(axis=1)
            new = rand_unit(chains)
            dE = -J * ((new - s[:, i, :]) * h).sum(axis=1)
            acc = rng.random(chains) < np.exp(np.minimum(0.0, -dE / T))
            s[acc, i, :] = new[acc]
        if sw >= discard:
            E = -J * (s[:, a, :] * s[:, b, :]).sum(axis=(1, 2))
            M = s.sum(axis=1)
            m2 = (M * M).sum(axis=1) / N ** 2
            E_samples.append(E.mean())
            m2_samples.append(m2.mean())
    E_arr = np.array(E_samples)
    m2_arr = np.array(m2_samples)
    # Chains are independent; sweeps within a chain are correlated, so use
    # bins over sweeps of the chain average.
    return binned_mean(E_arr, 20), binned_mean(m2_arr, 20)
