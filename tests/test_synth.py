"""Input generators: determinism, ranges and structure (no GPU)."""
import numpy as np

import synth


def test_uniform_deterministic_and_range():
    a = synth.uniform(100, seed=3)
    b = synth.uniform(100, seed=3)
    c = synth.uniform(100, seed=4)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert a.min() >= -1.0 and a.max() < 1.0
    assert a.flags.f_contiguous
    assert abs(a.mean()) < 0.02 and abs(a.var() - 1 / 3) < 0.02


def test_lda_padding_sentinel():
    a = synth.uniform(10, seed=1, lda=13)
    assert a.shape == (10, 10) and a.strides == (8, 13 * 8)
    assert np.array_equal(a, synth.uniform(10, seed=1))
    assert np.isnan(a.base[10:, :]).all()


def test_dominant_structure():
    a = synth.dominant(64, seed=2)
    off = np.abs(a).sum(axis=1) - np.abs(np.diag(a))
    assert (np.diag(a) > off).all()


def test_planted_structure():
    A, L, U, perm = synth.planted(32, seed=1)
    assert np.allclose(np.diag(L), 1.0) and np.abs(np.tril(L, -1)).max() < 0.1
    assert (np.diag(U) >= 1.0).all() and (np.diag(U) < 2.0).all()
    assert np.array_equal(np.sort(perm), np.arange(32))
    assert np.allclose(A[perm, :], L @ U)
