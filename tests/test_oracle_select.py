"""Pins for the selection oracle: features against brute force and
constructed cases, the interpolation fit against known polynomials."""
import numpy as np
import pytest

import oracle
from oracle import select as S
from paper_1801_01134_amd import synth


def _brute_features(A):
    n, m = A.n_rows, A.n_cols
    lens = [int(A.rowptr[i + 1] - A.rowptr[i]) for i in range(n)]
    nnz = sum(lens)
    mean = nnz / n
    f = [np.log2(n), np.log2(m), np.log2(nnz + 1), mean,
         (np.sqrt(sum((L - mean) ** 2 for L in lens) / n) / mean) if mean else 0.0,
         np.log2(1 + max(lens)), sum(1 for L in lens if L == 0) / n]
    dist = [abs(int(A.colidx[p]) - i) for i in range(n) for p in range(A.rowptr[i], A.rowptr[i + 1])]
    f.append(sum(dist) / len(dist) / max(n, m))
    for (r, c) in oracle.SHAPES:
        nb = 0
        for t in range((n + r - 1) // r):
            cols = [int(A.colidx[p]) for i in range(t * r, min(n, t * r + r))
                    for p in range(A.rowptr[i], A.rowptr[i + 1])]
            nb += oracle.min_cover_bruteforce(cols, c)
        f.append(nnz / nb)
    return np.array(f)


@pytest.mark.parametrize("seed", range(4))
def test_features_against_bruteforce(seed):
    A = synth.random_small(11, 19, 0.25, seed=seed)
    if A.nnz == 0:
        pytest.skip("empty draw")
    f = S.features(A)
    assert np.allclose(f[:14], _brute_features(A), rtol=1e-12, atol=1e-12)


def test_single_value_block_share_constructed():
    # entries 8 apart: every beta(1,8) block holds one value
    a = np.zeros((4, 64))
    a[:, ::8] = 1.0
    assert S.features(synth.from_dense(a))[14] == 1.0
    # dense rows: no single-value block
    assert S.features(synth.from_dense(np.ones((3, 16))))[14] == 0.0
    # row 0: one full block + one single; row 1: two singles -> 3 of 4 blocks
    b = np.zeros((2, 32))
    b[0, 0:8] = 1
    b[0, 20] = 1
    b[1, 3] = 1
    b[1, 30] = 1
    assert S.features(synth.from_dense(b))[14] == 0.75
    # span feature: contiguous rows span exactly their length -> log2(1) = 0
    assert S.features(synth.from_dense(np.ones((3, 16))))[15] == 0.0


def test_span_feature_constructed():
    # feature 15 = mean over non-empty rows of log2((last - first + 1) / length)
    #   row 0: columns {0, 7}        span 8, length 2 -> log2(4) = 2
    #   row 1: columns {3, 4, 5, 6}  span 4, length 4 -> 0
    #   row 2: empty (not counted)
    #   row 3: column {10}           span 1, length 1 -> 0
    #   row 4: columns {1, 2, 9, 16} span 16, length 4 -> log2(4) = 2
    # mean = (2 + 0 + 0 + 2) / 4 = 1; the inverted ratio would give -1, a span
    # without the + 1 log2(7/2) + log2(3/4) + ... != 1
    a = np.zeros((5, 20))
    for i, cols in enumerate([[0, 7], [3, 4, 5, 6], [], [10], [1, 2, 9, 16]]):
        a[i, cols] = 1.0
    assert S.features(synth.from_dense(a))[15] == 1.0
    # one row of length 3 spread over 12 columns: log2(12 / 3) = 2
    b = np.zeros((1, 12))
    b[0, [0, 5, 11]] = 1.0
    assert S.features(synth.from_dense(b))[15] == 2.0


def test_interpolation_recovers_known_cubic():
    rng = synth.rng_for(3)
    avgs = rng.uniform(1, 30, size=(40, 6))
    true = [np.array([0.001 * k, -0.03, 0.4 + 0.1 * k, 1.0 + k]) for k in range(6)]
    speeds = np.stack([np.polyval(true[k], avgs[:, k]) for k in range(6)], axis=1)
    model = S.fit_interpolation(avgs, speeds, degree=3)
    for k in range(6):
        assert np.allclose(model.coeffs[k], true[k], rtol=1e-8, atol=1e-10)
    q = np.array([5.0, 6, 7, 8, 9, 10])
    pred = model.predict(q)
    assert np.allclose(pred, [np.polyval(true[k], q[k]) for k in range(6)])
    assert model.select(q) == int(np.argmax(pred))
    # outside the fitted range the prediction is held at the range edge
    far = np.full(6, 1e6)
    assert np.allclose(model.predict(far), [np.polyval(true[k], avgs[:, k].max()) for k in range(6)])


def test_select_ties_take_lowest_index_and_regret():
    m = S.Interpolation([np.array([1.0])] * 6, np.zeros(6), np.ones(6), 0)
    assert m.select(np.zeros(6)) == 0
    t = np.array([2.0, 1.0, 1.5, 4.0, 1.0, 3.0])
    assert S.best_kernel(t) == 1
    assert S.regret(t, 1) == 0.0 and S.regret(t, 4) == 0.0
    assert S.regret(t, 0) == pytest.approx(1.0)


def test_interpolation_2d_recovers_a_known_surface():
    # speed_k(Avg, u) = sum c_k[i, j] Avg^i u^j exactly, u = log2 share in {-3..0}
    rng = synth.rng_for(4)
    n = 200
    avgs = rng.uniform(1, 30, size=(n, 6))
    u = rng.choice([-3.0, -2.0, -1.0, 0.0], size=n)
    true = [rng.normal(size=(4, 3)) * np.array([[1.0], [0.1], [0.01], [0.001]]) for _ in range(6)]
    speeds = np.stack([sum(true[k][i, j] * avgs[:, k] ** i * u ** j for i in range(4) for j in range(3))
                       for k in range(6)], axis=1)
    m = S.fit_interpolation_2d(avgs, u, speeds, 3, 2)
    for k in range(6):
        assert np.allclose(m.coeffs[k], true[k], rtol=1e-7, atol=1e-9)
    q = np.full(6, 7.0)
    for share in (0.125, 0.5, 1.0):
        want = [sum(true[k][i, j] * 7.0 ** i * np.log2(share) ** j for i in range(4) for j in range(3))
                for k in range(6)]
        assert np.allclose(m.predict(q, share), want)
        assert m.select(q, share) == int(np.argmax(want))
    # shares outside the fitted range are held at its edge
    assert np.allclose(m.predict(q, 1e-3), m.predict(q, 0.125))


def test_interpolation_2d_with_one_share_is_the_1d_fit():
    # records taken at one share only: the share degree drops to 0 and the
    # fit is the per-kernel polynomial of the sequential method
    rng = synth.rng_for(5)
    avgs = rng.uniform(1, 20, size=(60, 6))
    speeds = rng.uniform(1, 5, size=(60, 6))
    m2 = S.fit_interpolation_2d(avgs, np.zeros(60), speeds, 3, 2)
    m1 = S.fit_interpolation(avgs, speeds, 3)
    for k in range(6):
        assert m2.coeffs[k].shape == (4, 1)
        assert np.allclose(m2.coeffs[k][:, 0], m1.coeffs[k][::-1], rtol=1e-8, atol=1e-10)
    q = rng.uniform(1, 20, size=6)
    assert np.allclose(m2.predict(q, 1.0), m1.predict(q))
