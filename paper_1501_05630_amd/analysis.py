"""Host post-processing of the library's readouts (no simulation step runs here).

The paper's observables are formed on the device (icm_read_observables sums
E_a + E_b, N_b q_l, q^2 and the potential cluster sites per logarithmic time
bin); these helpers turn the sums into the quantities the paper plots:
E(q_l) and Delta of Eq. 1 and Eq. 2 ("Benchmark model and observables"), the
fraction p of potential cluster sites (the first figure's quantity), a
reproducible reading of the thermalization time (the third figure's quantity),
and the percolation Binder ratio with its finite-size-scaling collapse
(Supplemental Material).
"""
import numpy as np

# observable field 0 (E_a + E_b) for float couplings is in units of 2^-20
OBS_ENERGY_UNIT_FLOAT = 2.0 ** -20


def delta_per_bin(sums, counts, temps, n_sites, n_bonds, energy_unit):
    """Eq. 1 and 2 from the observable sums of one instance (icm_read_observables):
    returns (e_ql, e, delta) arrays [bins][K], averaged over the replica pairs:
    e_ql = E(q_l) = -(1/T)(N_b/N)(1 - q_l) for unit-variance couplings, e = <H/N>,
    delta = e_ql - e.  Bins without samples are NaN."""
    sums = np.asarray(sums, dtype=np.float64)
    c = np.asarray(counts, dtype=np.float64)[:, None]
    with np.errstate(invalid="ignore", divide="ignore"):
        ql = sums[:, :, :, 1].mean(axis=2) / (n_bonds * c)
        e = sums[:, :, :, 0].mean(axis=2) * energy_unit / (2.0 * n_sites * c)
        e_ql = -(1.0 / np.asarray(temps, dtype=np.float64))[None, :] * (n_bonds / n_sites) * (1.0 - ql)
    return e_ql, e, e_ql - e


def cluster_fraction_per_bin(sums, counts, n_sites):
    """The fraction p of potential cluster sites (sites of negative overlap after
    step 2a) per time bin and temperature, [bins][K], averaged over the replica
    pairs, from the observable sums of one instance.  Bins without samples are
    NaN."""
    sums = np.asarray(sums, dtype=np.float64)
    c = np.asarray(counts, dtype=np.float64)[:, None]
    with np.errstate(invalid="ignore", divide="ignore"):
        return sums[:, :, :, 3].mean(axis=2) / (n_sites * c)


def thermalization_bin(mean, se, complete, n_se=2.0):
    """First time bin from which a disorder-averaged Delta stays at zero: the
    smallest b such that every complete bin b' >= b has |mean[b']| <= n_se
    se[b'] (the paper deems a system thermalized once Delta ~ 0 and read the
    times off by eye).  None if the last complete bin is not at zero yet."""
    bins = [b for b in range(len(mean)) if complete[b]]
    first = None
    for b in reversed(bins):
        if abs(mean[b]) <= n_se * se[b]:
            first = b
        else:
            break
    return first


def binder_ratio(smax):
    """g = (3 - <s^4> / <s^2>^2) / 2 of the largest-cluster sizes of a set of
    random configurations (the percolation Binder ratio of the Supplemental
    Material; 1 when every configuration has the same s_max)."""
    s = np.asarray(smax, dtype=np.float64)
    m2, m4 = np.mean(s ** 2), np.mean(s ** 4)
    return 0.5 * (3.0 - m4 / (m2 * m2))


def binder_collapse(ps, sizes, g, se, p_c0, nu0, degree=3):
    """Finite-size scaling of the percolation Binder ratio, g(p, N) =
    G[N^(1/(2 nu)) (1/p - 1/p_c)] (the scaling form of the Supplemental
    Material with sqrt(N) as the linear size): the (p_c, nu) for which one
    polynomial of the scaling variable fits every size's curve best, by
    weighted least squares.  ps [P]; sizes [S] (site counts N); g, se [S][P].
    Returns (p_c, nu, chi2 per degree of freedom)."""
    from scipy.optimize import minimize
    ps = np.asarray(ps, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    se = np.asarray(se, dtype=np.float64)

    def chi2(theta):
        pc, nu = theta
        if not (0 < pc < 1 and nu > 0.05):
            return 1e30
        x = np.concatenate([n ** (0.5 / nu) * (1.0 / ps - 1.0 / pc) for n in sizes])
        y, w = g.reshape(-1), 1.0 / se.reshape(-1)
        c = np.polyfit(x, y, degree, w=w)
        return float(np.sum(((np.polyval(c, x) - y) * w) ** 2))

    best = minimize(chi2, [p_c0, nu0], method="Nelder-Mead",
                    options={"xatol": 1e-7, "fatol": 1e-9, "maxiter": 4000})
    dof = g.size - (degree + 1) - 2
    return float(best.x[0]), float(best.x[1]), best.fun / max(dof, 1)
