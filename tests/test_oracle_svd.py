"""Oracle pins for the block-wise SVD, its global truncation and the
block-wise symmetric eigen-decomposition.

Pinned against the dense matrix of the same tensor (rows = the first two
legs): its singular values are the union of the sector values, each SU(2)
sector's values repeated 2e + 1 times; the truncation's discarded weight is
the dense tail beyond the kept count (Eckart-Young); the eigenvalues of its
symmetric part are the union of the sectors' eigenvalues.  The symmetric part
itself is pinned by the closed-form spectrum of a tridiagonal Toeplitz
matrix."""
import numpy as np
import pytest

import workloads as W
from oracle import svd as SV
from oracle import tensors as T


def _dense_matrix(spec, flat, n_row=2):
    d = T.to_dense(spec, flat)
    r = int(np.prod(d.shape[:n_row]))
    return d.reshape(r, -1)


def _spectrum(values, spec):
    out = []
    for s, v in values.items():
        out += list(v) * SV.multiplicity(spec, s)
    return np.sort(np.array(out))[::-1]


def _u1_cases():
    c1 = W.config1().A
    li = W.u1_leg(-2, 2, [1, 2, 3, 2, 1], W.IN)
    lo = W.u1_leg(-1, 1, [2, 3, 2], W.OUT)
    cov = W.TensorSpec(W.U1, (li, li, lo, lo), qtot=1)      # sectors of unequal rows and columns
    return [c1, cov]


@pytest.mark.parametrize("k", [0, 1])
def test_u1_block_values_are_the_dense_spectrum(k):
    spec = _u1_cases()[k]
    flat = np.random.default_rng(k).standard_normal(T.num_elements(spec))
    vals = SV.block_singular_values(spec, flat, 2)
    mats = SV.sector_matrices(spec, flat, 2)
    assert any(m.shape[0] < m.shape[1] for m in mats.values()) or k == 0
    assert any(m.shape[0] > m.shape[1] for m in mats.values()) or k == 0
    dense = np.linalg.svd(_dense_matrix(spec, flat), compute_uv=False)
    blocks = _spectrum(vals, spec)
    np.testing.assert_allclose(dense[:blocks.size], blocks, rtol=1e-12, atol=1e-12)
    assert np.all(np.abs(dense[blocks.size:]) < 1e-12)


def test_su2_values_repeat_2e_plus_1_times():
    spec = W.su2_pair(2, [2, 1, 2])[0]          # OPERATOR tree, spins 0, 1/2, 1
    flat = np.random.default_rng(3).standard_normal(T.num_elements(spec))
    vals = SV.block_singular_values(spec, flat, 2)
    dense = np.linalg.svd(_dense_matrix(spec, flat), compute_uv=False)
    blocks = _spectrum(vals, spec)
    np.testing.assert_allclose(dense[:blocks.size], blocks, rtol=1e-12, atol=1e-12)
    assert np.all(np.abs(dense[blocks.size:]) < 1e-12)
    # weighting by 1 (a planted mistake) would not reproduce the dense spectrum
    flat_only = np.sort(np.concatenate(list(vals.values())))[::-1]
    assert flat_only.size < blocks.size


@pytest.mark.parametrize("which", ["u1", "su2"])
def test_truncation_discards_the_dense_tail(which):
    spec = _u1_cases()[0] if which == "u1" else W.su2_pair(2, [2, 1, 2])[0]
    flat = np.random.default_rng(4).standard_normal(T.num_elements(spec))
    vals = SV.block_singular_values(spec, flat, 2)
    dense = np.linalg.svd(_dense_matrix(spec, flat), compute_uv=False)
    for chi in (1, 7, 20, 10 ** 6):
        keep, lost = SV.truncate(spec, vals, chi)
        used = sum(SV.multiplicity(spec, s) * n for s, n in keep.items())
        assert used <= chi
        np.testing.assert_allclose(lost, float(np.sum(dense[used:] ** 2)), rtol=1e-10, atol=1e-12)
        if chi >= dense.size:
            assert lost < 1e-20


def test_symmetric_part_of_tridiagonal_toeplitz():
    # diagonal a, superdiagonal b + d, subdiagonal b - d: the symmetric part is
    # the Toeplitz matrix (a, b), eigenvalues a + 2 b cos(k pi / (n + 1))
    n, a, b, d = 37, 0.3, -1.25, 0.8
    m = a * np.eye(n) + (b + d) * np.eye(n, k=1) + (b - d) * np.eye(n, k=-1)
    ref = np.sort(a + 2 * b * np.cos(np.arange(1, n + 1) * np.pi / (n + 1)))[::-1]
    np.testing.assert_allclose(SV.symmetric_eigenvalues(m), ref, rtol=0, atol=1e-13)
    # the lower triangle alone (a planted mistake) gives the (a, b - d) spectrum
    wrong = np.linalg.eigvalsh(m)[::-1]
    assert np.max(np.abs(wrong - ref)) > 0.5
    with pytest.raises(ValueError):
        SV.symmetric_eigenvalues(np.zeros((3, 4)))


@pytest.mark.parametrize("which", ["u1", "su2"])
def test_block_eigenvalues_are_the_dense_spectrum(which):
    spec = W.config1().A if which == "u1" else W.su2_pair(2, [2, 1, 2])[0]
    flat = np.random.default_rng(5).standard_normal(T.num_elements(spec))
    vals = SV.block_eigenvalues(spec, flat, 2)
    d = _dense_matrix(spec, flat)
    assert d.shape[0] == d.shape[1]
    dense = np.linalg.eigvalsh(0.5 * (d + d.T))[::-1]
    blocks = _spectrum(vals, spec)
    # every dense row lies in one sector, so nothing is left over
    assert blocks.size == dense.size
    np.testing.assert_allclose(dense, blocks, rtol=0, atol=1e-12 * np.abs(dense).max())


@pytest.mark.parametrize("shape", [(9, 6), (6, 9), (7, 7)])
def test_polar_factors_of_a_built_matrix(shape):
    # m = Qa diag(s) Qb^T with orthonormal Qa, Qb: the polar factor is
    # Qa Qb^T and the positive factor Qb diag(s) Qb^T (rows >= columns) or
    # Qa diag(s) Qa^T
    rng = np.random.default_rng(11)
    M, N = shape
    k = min(M, N)
    qa, _ = np.linalg.qr(rng.standard_normal((M, k)))
    qb, _ = np.linalg.qr(rng.standard_normal((N, k)))
    s = np.linspace(3.0, 0.5, k)
    m = (qa * s) @ qb.T
    w, p = SV.polar_factors(m)
    np.testing.assert_allclose(w, qa @ qb.T, atol=1e-13)
    pref = (qb * s) @ qb.T if M >= N else (qa * s) @ qa.T
    np.testing.assert_allclose(p, pref, atol=1e-13)
    np.testing.assert_allclose(w @ p if M >= N else p @ w, m, atol=1e-13)
    # a transposed right factor (a planted mistake) is not the polar factor
    if M == N:
        u, _, vt = np.linalg.svd(m)
        assert np.abs(u @ vt.T - qa @ qb.T).max() > 1e-3


def test_polar_of_a_scalar_is_its_sign_and_size():
    w, p = SV.polar_factors(np.array([[-3.0]]))
    assert w[0, 0] == pytest.approx(-1.0) and p[0, 0] == pytest.approx(3.0)


def test_block_polar_rebuilds_every_sector():
    spec = _u1_cases()[1]          # sectors of unequal rows and columns
    flat = np.random.default_rng(6).standard_normal(T.num_elements(spec))
    mats = SV.sector_matrices(spec, flat, 2)
    for sec, (w, p) in SV.block_polar(spec, flat, 2).items():
        m = mats[sec]
        np.testing.assert_allclose(w @ p if m.shape[0] >= m.shape[1] else p @ w, m, atol=1e-12)
        np.testing.assert_allclose(p, p.T, atol=1e-13)
