"""Pins of the oracle's sampled leverage-score selection (Algorithm 3 as stated) and of its
counter-based generator, on the CPU:

  * Philox4x32-10 against the known-answer vectors published with the generator (Random123);
  * the 53-bit uniforms: range, mean and variance, and independent streams per pass and side;
  * the selection's inclusion frequencies over many keys against p_i = min(1, rho pi_i)
    (a wrong probability, a dropped factor or an inverted comparison fails this);
  * the selection against a plain loop written from the definition, including the cap and the
    safeguard's random index.
"""
import math

import numpy as np
import pytest

from oracle import crossdeim as cd


@pytest.mark.parametrize("ctr,key,want", [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
])
def test_philox_known_answers(ctr, key, want):
    out = cd.philox4x32_10(*[np.array([c], dtype=np.uint64) for c in ctr], *key)
    assert tuple(int(x[0]) for x in out) == want


def test_uniforms_are_uniform_and_streams_independent():
    n = 200_000
    u = cd.sample_uniforms(n, 3, 0, 12345)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 4 * math.sqrt(1 / 12 / n)
    assert abs(u.var() - 1 / 12) < 0.002
    # histogram of 20 bins within 5 sigma of n / 20
    h, _ = np.histogram(u, bins=20, range=(0.0, 1.0))
    assert np.all(np.abs(h - n / 20) < 5 * math.sqrt(n / 20))
    for other in (cd.sample_uniforms(n, 4, 0, 12345), cd.sample_uniforms(n, 3, 1, 12345),
                  cd.sample_uniforms(n, 3, 0, 12346)):
        assert abs(np.corrcoef(u, other)[0, 1]) < 5 / math.sqrt(n)
    # the same counters give the same numbers
    assert np.array_equal(u, cd.sample_uniforms(n, 3, 0, 12345))


def _orthonormal(n, r, seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((n, r)))
    return q


def test_inclusion_frequency_is_min_one_rho_pi():
    n, r, rho = 40, 3, 6.0
    U = _orthonormal(n, r, 1)
    U[5] /= np.linalg.norm(U[5])  # one row with score 1, so p = 1
    I_prev = [0, 7, 9]
    score = np.sum(U[:, :r] ** 2, axis=1)
    p = np.minimum(1.0, rho * score)
    trials = 3000
    count = np.zeros(n)
    for seed in range(trials):
        u = cd.sample_uniforms(n, 0, 0, seed)
        sel = cd.sampled_select(U, r, I_prev, n, rho, u)
        for i in sel.new:
            count[i] += 1
    freq = count / trials
    free = np.ones(n, dtype=bool)
    free[I_prev] = False
    sd = np.sqrt(p * (1 - p) / trials) + 1e-12
    # a safeguard pick (when nothing is kept) adds at most P(nothing kept) to a frequency
    none = np.prod(1 - p[free])
    assert np.all(np.abs(freq[free] - p[free]) <= 5 * sd[free] + none)
    assert np.all(freq[~free] == 0.0)
    assert freq[5] == 1.0


def _loop_select(U, r_sig, I_prev, p_max, rho, u):
    n = U.shape[0]
    pi = [sum(U[i, e] ** 2 for e in range(r_sig)) for i in range(n)]
    top = max(pi)
    score = [0.0 if x <= cd.FLOOR_REL * top else x for x in pi]
    kept = [i for i in range(n) if i not in I_prev and u[i] < min(1.0, rho * score[i])]
    kept.sort(key=lambda i: (-score[i], i))
    room = max(0, min(p_max, n) - len(I_prev))
    new = sorted(kept[:room])
    if not new and room > 0:
        free = [i for i in range(n) if i not in I_prev]
        free.sort(key=lambda i: (-(-1.0 - u[i]), i))
        new = [free[0]]
    return list(I_prev) + new


@pytest.mark.parametrize("case", range(12))
def test_selection_equals_a_plain_loop(case):
    rng = np.random.default_rng(100 + case)
    n, r = int(rng.integers(8, 60)), int(rng.integers(1, 5))
    U = _orthonormal(n, r, case)
    if case % 3 == 0:
        U[rng.integers(0, n, 3)] = 0.0  # rows at the noise floor
    I_prev = sorted(rng.choice(n, int(rng.integers(0, n // 3)), replace=False).tolist())
    rho = [0.01, 1.0, 4.0, 50.0][case % 4]  # 0.01: usually nothing kept (the safeguard)
    p_max = int(rng.integers(len(I_prev), n + 1))
    u = cd.sample_uniforms(n, case, case % 2, 99)
    got = cd.sampled_select(U, r, I_prev, p_max, rho, u).indices
    assert got == _loop_select(U, r, I_prev, p_max, rho, u)


def test_sampled_solve_pins():
    """A whole sampled solve on a small grid: deterministic for a key, different for another,
    and within 100 times the best rank-16 error of the dense DST solution (Eckart-Young)."""
    import workloads
    from oracle import dense

    n = 63
    U, s, V = workloads.make("n255_r5_fp64", 0, n=n)
    a = cd.solve(n, U, s, V, 16, 1e-10, 20, selector="ls_sampled", ls_oversampling=3.0, seed=5)
    b = cd.solve(n, U, s, V, 16, 1e-10, 20, selector="ls_sampled", ls_oversampling=3.0, seed=5)
    c = cd.solve(n, U, s, V, 16, 1e-10, 20, selector="ls_sampled", ls_oversampling=3.0, seed=6)
    assert [t.I_pre for t in a.trace] == [t.I_pre for t in b.trace]
    assert [t.I_pre for t in a.trace] != [t.I_pre for t in c.trace]
    W = dense.dense_solve((U * s[None, :]) @ V.T)
    Wa = (a.U * a.S[None, :]) @ a.V.T
    sv = np.linalg.svd(W, compute_uv=False)
    best = math.sqrt(float(np.sum(sv[16:] ** 2)))
    assert np.linalg.norm(Wa - W) <= 100.0 * best
