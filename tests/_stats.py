"""The statistical bar for time averages of chaotic trajectories (shared by
the GPU tests that compare averages with oracle runs).

z = |a_gpu - a_oracle| / hypot(se_gpu, se_oracle), each SE from 10 blocks
(9 degrees of freedom each). Under the null hypothesis P(z > 3) is about
0.8 % (close to Student's t with 18 degrees of freedom, checked by
simulation), so the number of z above 3 among n values is binomial; a check
allows the largest count whose binomial tail is still above 1e-3 and no z
above 5. A systematic offset (a missing term, a wrong factor) shows up as a
signed mean of z over the sample; that mean must stay within 4 / sqrt(n).
"""
import math

import numpy as np
import pytest

P_OVER3 = 0.0078  # P(z > 3) for the statistic above under the null


def max_exceedances(n, p=P_OVER3, level=1e-3):
    """Largest count k with P(Binomial(n, p) > k) still above level, plus one."""
    from scipy import stats
    k = 0
    while stats.binom.sf(k, n, p) > level:
        k += 1
    return k


def check_stats(g, o, what, labels=None, failed_mask=(1 | 8), ecold_abs=None):
    """g: device results; o: oracle tuples (P, P_se, T, T_se, Ecold per atom).
    E_cold per atom must match to 1e-6 relative, or, where ecold_abs gives a
    per-cell absolute bar (terms that cancel), to within that bar."""
    zs = []  # signed, per cell: (P, T)
    for k, (gi, (P, Pse, T, Tse, Ec)) in enumerate(zip(g, o)):
        assert gi["status"] & failed_mask == 0
        if ecold_abs is None:
            assert gi["Ecold"] == pytest.approx(Ec, rel=1e-6)
        else:
            assert abs(gi["Ecold"] - Ec) <= ecold_abs[k], (k, gi["Ecold"], Ec, ecold_abs[k])
        zs.append(((gi["P"] - P) / math.hypot(gi["P_se"], Pse), (gi["T"] - T) / math.hypot(gi["T_se"], Tse)))
    zs = np.array(zs)
    z = np.abs(zs).ravel()
    n = len(g)
    kmax = max_exceedances(z.size)
    print(f"{what}: {n} cells, max z {z.max():.2f}, over 3: {(z > 3).sum()} (allowed {kmax}), "
          f"mean signed z P {zs[:, 0].mean():+.2f} T {zs[:, 1].mean():+.2f}", flush=True)
    for i in range(n):
        print(f"  {labels[i] if labels else i}: zP {zs[i, 0]:+.2f} zT {zs[i, 1]:+.2f}", flush=True)
    assert (z > 3).sum() <= kmax and z.max() <= 5, zs
    assert abs(zs[:, 0].mean()) <= 4 / math.sqrt(n) and abs(zs[:, 1].mean()) <= 4 / math.sqrt(n), zs


def _oracle_job(args):
    import oracle
    cell, n, na, resc = args
    r = oracle.run(cell, oracle.Schedule(n, na, rescale_steps=tuple(resc))).result
    return r.P, r.P_se, r.T, r.T_se, r.Ecold


def oracle_many(cells, n_steps, n_avg, rescale_steps, workers=16):
    """Oracle runs of many cells in parallel processes (one cell each), with
    the default block count and energy sampling of both sides."""
    import multiprocessing as mp
    jobs = [(c, n_steps, n_avg, list(rescale_steps)) for c in cells]
    with mp.get_context("fork").Pool(min(workers, max(1, len(jobs)))) as pool:
        return pool.map(_oracle_job, jobs, chunksize=1)
