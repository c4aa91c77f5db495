"""Pins of the Bloch (k-point) operator in the phase-twisted form.

* k = 0 through the complex code path equals the real path;
* time reversal: with a real potential, spectrum(k) = spectrum(-k);
* the twisted operator is Hermitian and the Bloch phases have unit modulus;
* k and k + 2 pi / L e_x give the same spectrum (Bloch periodicity in k).
"""
import numpy as np
import pytest

from oracle.operator import OEFEOperator
from paper_2010_09701_amd import workloads as wl


def _sys():
    return wl.tiny_system(nc=3, p=2, n_atoms=2, seed=13, L=6.0, r0=1.0, r1=2.3)


def test_k_zero_complex_equals_real():
    s = _sys()
    Hr = OEFEOperator(s).dense()
    Hc = OEFEOperator(s.with_k(np.zeros(3))).dense()
    assert Hc.dtype == np.complex128
    np.testing.assert_allclose(Hc, Hr, atol=1e-12 * np.abs(Hr).max())


def test_time_reversal_and_hermitian():
    s = _sys()
    k = np.array([0.25, -0.1, 0.4])
    Hp = OEFEOperator(s.with_k(k)).dense()
    Hm = OEFEOperator(s.with_k(-k)).dense()
    assert np.abs(Hp - np.conj(Hp.T)).max() < 1e-13 * np.abs(Hp).max()
    np.testing.assert_allclose(np.linalg.eigvalsh(Hp), np.linalg.eigvalsh(Hm), atol=1e-11 * np.abs(Hp).max())
    # time reversal also means H(-k) = conj(H(k))
    np.testing.assert_allclose(Hm, np.conj(Hp), atol=1e-12 * np.abs(Hp).max())


def test_phase_modulus_and_reciprocal_lattice_periodicity():
    s = _sys()
    k = np.array([0.25, -0.1, 0.4])
    op = OEFEOperator(s.with_k(k))
    np.testing.assert_allclose(np.abs(op.theta), 1.0, atol=1e-15)
    G = np.array([2 * np.pi / s.L, 0, 0])
    l1 = np.linalg.eigvalsh(op.dense())
    l2 = np.linalg.eigvalsh(OEFEOperator(s.with_k(k + G)).dense())
    np.testing.assert_allclose(l1, l2, atol=1e-10 * np.abs(l1).max())
