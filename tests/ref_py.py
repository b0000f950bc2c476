"""Independent set-based restatement of RSAI(tol) for tiny dense matrices.

Written separately from the C oracle, in plain Python sets and numpy, with the LS
problem (2.3) solved by ``numpy.linalg.lstsq`` and the residual (2.4) formed on all n
rows. It is a brute-force cross-check of the oracle's index logic (Algorithm 1 and
the dropping of Section 4) on n <= 64, not a second product implementation.
"""
import numpy as np


def rsai_dense(Ad, c=3, lmax=8, eps=0.4, drop=1, tol=1e-3):
    n = Ad.shape[0]
    norm1 = np.abs(Ad).sum(axis=0).max()
    rowpat = [set(np.nonzero(Ad[i, :])[0].tolist()) for i in range(n)]
    colpat = [set(np.nonzero(Ad[:, j])[0].tolist()) for j in range(n)]
    cols = []
    for k in range(n):
        ek = np.zeros(n)
        ek[k] = 1.0

        def solve(I, J):
            Is, Js = sorted(I), sorted(J)
            x = np.linalg.lstsq(Ad[np.ix_(Is, Js)], ek[Is], rcond=None)[0]
            r = Ad[:, Js] @ x - ek
            return dict(zip(Js, x)), r

        def dropped(I, J, m, r):
            if drop == 0:
                return J, m, r
            t = tol if drop == 1 else eps / (len(J) * norm1)
            keep = {j for j in J if abs(m[j]) > t}
            if keep == J:
                return J, m, r
            if not keep:
                best = max(sorted(J), key=lambda j: abs(m[j]))
                keep = {best}
            m, r = solve(I, keep)
            return keep, m, r

        J = {k}
        I = set(colpat[k])
        R = set()
        l = 0
        m, r = solve(I, J)
        J, m, r = dropped(I, J, m, r)
        while np.linalg.norm(r) > eps and l < lmax:
            cand = [i for i in range(n) if r[i] != 0.0 and i not in R]
            if not cand:
                break
            cand.sort(key=lambda i: (-abs(r[i]), i))
            Rh = cand[:c]
            R |= set(Rh)
            Jh = set().union(*(rowpat[i] for i in Rh)) - J
            l += 1
            if not Jh:
                continue
            Ih = set().union(*(colpat[j] for j in Jh)) - I
            J |= Jh
            I |= Ih
            m, r = solve(I, J)
            J, m, r = dropped(I, J, m, r)
        cols.append((sorted(J), [m[j] for j in sorted(J)], l, np.linalg.norm(r), len(I)))
    return cols
