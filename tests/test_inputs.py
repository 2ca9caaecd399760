"""Seeded input generators: SU(3) membership, Haar moments, determinism."""

import numpy as np
import pytest

from paper_1311_2719_amd import inputs


def _su3_errors(U):
    M = U.reshape(-1, 3, 3)
    eye = np.eye(3)
    unit = np.max(np.abs(np.conj(np.swapaxes(M, -1, -2)) @ M - eye))
    det = np.max(np.abs(np.linalg.det(M) - 1.0))
    return unit, det


def test_haar_is_su3():
    U = inputs.haar_su3((4, 4, 4, 4), seed=101)
    assert U.shape == (256, 4, 3, 3) and U.dtype == np.complex128
    unit, det = _su3_errors(U)
    assert unit < 1e-13 and det < 1e-13


def test_haar_moments():
    # Haar measure on SU(3): E[tr U] = 0, E[|tr U|^2] = 1, E[|U_ij|^2] = 1/3.
    U = inputs.haar_su3((8, 8, 8, 8), seed=7).reshape(-1, 3, 3)
    n = U.shape[0]
    tr = np.trace(U, axis1=-2, axis2=-1)
    # tr U has unit second moment, so its mean has std 1/sqrt(2n) per component
    assert abs(tr.mean()) < 5.0 / np.sqrt(n)
    m2 = np.mean(np.abs(tr) ** 2)
    assert abs(m2 - 1.0) < 5.0 * np.std(np.abs(tr) ** 2) / np.sqrt(n)
    e = np.abs(U) ** 2
    assert np.all(np.abs(e.mean(axis=0) - 1.0 / 3.0) < 5.0 * e.std(axis=0) / np.sqrt(n))


def test_smooth_is_su3_and_near_identity():
    U3 = inputs.smooth_su3((4, 4, 4, 4), eps=0.3, seed=102)
    U5 = inputs.smooth_su3((4, 4, 4, 4), eps=0.5, seed=102)
    for U in (U3, U5):
        unit, det = _su3_errors(U)
        assert unit < 1e-13 and det < 1e-13
    p3 = np.mean(np.real(np.trace(U3, axis1=-2, axis2=-1))) / 3
    p5 = np.mean(np.real(np.trace(U5, axis1=-2, axis2=-1))) / 3
    assert 1.0 > p3 > p5 > 0.5


def test_smooth_chunking_is_invisible():
    a = inputs.smooth_su3((4, 4, 4, 2), eps=0.5, seed=3, chunk=1 << 18)
    b = inputs.smooth_su3((4, 4, 4, 2), eps=0.5, seed=3, chunk=37)
    assert np.array_equal(a, b)


def test_sources_and_seeds():
    a = inputs.gaussian_source((4, 4, 4, 4), 201)
    b = inputs.gaussian_source((4, 4, 4, 4), 201)
    c = inputs.gaussian_source((4, 4, 4, 4), 202)
    assert a.shape == (256, 3) and np.array_equal(a, b) and not np.array_equal(a, c)
    big = inputs.gaussian_source((8, 8, 8, 8), 5)
    assert abs(np.mean(np.abs(big) ** 2) - 2.0) < 0.05


def test_masses_uniform():
    m = inputs.masses_uniform(0.01, 0.2, 12)
    assert m[0] == 0.01 and m[-1] == 0.2 and len(m) == 12
    assert np.allclose(np.diff(m), (0.2 - 0.01) / 11)


def test_volume_rejects_bad_dims():
    with pytest.raises(ValueError):
        inputs.volume((4, 4, 4))
