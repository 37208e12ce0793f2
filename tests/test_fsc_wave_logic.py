"""The shell-sum kernel's wave logic (fsc_shell_kernel in pwf_tomo.hip), modelled lane by
lane on the CPU: for chunks of 64 lanes x K elements whose shell index is monotone (the
kernel's chunks lie in one half of an x row), the per-lane runs, the scan of the maps
x -> A x + B and the three kinds of histogram stores must give the per-shell sums of a
bincount, with the lanes of any one store writing distinct shells (no atomics needed)."""

from collections import defaultdict

import numpy as np
import pytest

LANES = 64


def wave_model(shells, vals, K, nsh):
    sk = shells.reshape(LANES, K)
    v = vals.reshape(LANES, K)
    h = np.zeros(nsh)
    stores = defaultdict(list)

    def put(ins, k, x):
        if k < nsh:
            stores[ins].append(k)
            h[k] += x

    f = np.zeros(LANES)
    q = np.zeros(LANES)
    sf = sk[:, 0].copy()
    sq = sk[:, 0].copy()
    multi = np.zeros(LANES, bool)
    for j in range(K):
        vj = np.where(sk[:, j] == nsh, 0.0, v[:, j])
        for lane in range(LANES):
            if j == 0:
                f[lane] = vj[lane]
            elif sk[lane, j] == sq[lane]:
                if multi[lane]:
                    q[lane] += vj[lane]
                else:
                    f[lane] += vj[lane]
            else:
                if multi[lane]:
                    put(("inner", j), sq[lane], q[lane])
                multi[lane] = True
                sq[lane] = sk[lane, j]
                q[lane] = vj[lane]
    sl = np.where(multi, sq, sf)
    join = np.array([lane > 0 and sl[lane - 1] == sf[lane] for lane in range(LANES)])
    A = (~multi & join).astype(int)
    B = np.where(multi, q, f).astype(float)
    d = 1
    while d < LANES:
        Ap, Bp = A.copy(), B.copy()
        for lane in range(d, LANES):
            if A[lane]:
                B[lane] += Bp[lane - d]
            A[lane] &= Ap[lane - d]
        d *= 2
    for lane in range(LANES):
        if multi[lane]:
            put("first", sf[lane], f[lane] + (B[lane - 1] if join[lane] else 0.0))
    for lane in range(LANES):
        if not (lane < LANES - 1 and sf[lane + 1] == sl[lane]):
            put("last", sl[lane], B[lane])
    return h, stores


@pytest.mark.parametrize("K", [1, 4])
def test_wave_logic_matches_bincount(K):
    rng = np.random.default_rng(K)
    nsh = 40
    for trial in range(300):
        n = LANES * K
        steps = rng.choice([0, 0, 0, 1, 1, 2, 5], size=n) * (rng.random(n) < rng.random())
        s = np.cumsum(steps) + rng.integers(0, 10)
        if trial % 2:
            s = s[::-1]          # the half of the row with negative kx: kappa decreasing
        s = np.minimum(s, nsh)   # nsh marks elements outside the last shell
        v = rng.standard_normal(n)
        h, stores = wave_model(s, v, K, nsh)
        ref = np.bincount(s[s < nsh], v[s < nsh], nsh)
        assert np.allclose(h, ref, rtol=0, atol=1e-12)
        for ks in stores.values():
            assert len(ks) == len(set(ks))
