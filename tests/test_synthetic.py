"""The seeded input generators: the gauge links are SU(3) and equal the
exponential taken through the eigendecomposition of the same Hermitian H."""
import numpy as np

import synthetic as syn


def test_gauge_links_are_su3_exponentials_of_the_drawn_algebra():
    L, eps, seed = (4, 4, 2, 6), 0.3, 77
    U = syn.gauge_field(L, eps, seed)
    w = syn.rng(seed).standard_normal((int(np.prod(L)), 4, 8))
    H = np.einsum("vma,aij->vmij", w, syn.gell_mann() / 2.0)
    e, q = np.linalg.eigh(H)
    ref = (q * np.exp(1j * eps * e)[..., None, :]) @ np.conj(np.swapaxes(q, -1, -2))
    assert np.max(np.abs(U - ref)) < 1e-13
    assert np.max(np.abs(U @ np.conj(np.swapaxes(U, -1, -2)) - np.eye(3))) < 1e-14
    assert np.max(np.abs(np.linalg.det(U) - 1.0)) < 1e-14


def test_large_angle_and_gauge_transform():
    """The closed form holds at large eps (eigenvalue phases beyond pi) and for
    the gauge transformations (eps = 1.7)."""
    w = syn.rng(5).standard_normal((2000, 8))
    H = np.einsum("va,aij->vij", w, syn.gell_mann() / 2.0)
    for eps in (1.7, 4.0):
        e, q = np.linalg.eigh(H)
        ref = (q * np.exp(1j * eps * e)[..., None, :]) @ np.conj(np.swapaxes(q, -1, -2))
        assert np.max(np.abs(syn._su3_from_algebra(w, eps) - ref)) < 1e-12
    g = syn.random_gauge_transform((2, 2, 2, 2), 9)
    assert np.max(np.abs(g @ np.conj(np.swapaxes(g, -1, -2)) - np.eye(3))) < 1e-14


def test_device_generators_match_and_repeat():
    """gauge_field_device evaluates gauge_field's closed form on a torch device
    from the same draws (on the CPU device: identical values); the device start
    vectors repeat for a seed and differ across seeds."""
    a = syn.gauge_field((2, 2, 2, 4), 0.3, 17)
    b = syn.gauge_field_device((2, 2, 2, 4), 0.3, 17, "cpu")
    assert np.array_equal(a, b.numpy())
    v1 = syn.start_vectors_device(3, 16, 12, 5, "cpu")
    v2 = syn.start_vectors_device(3, 16, 12, 5, "cpu")
    v3 = syn.start_vectors_device(3, 16, 12, 6, "cpu")
    assert v1.shape == (3, 16, 12) and np.array_equal(v1.numpy(), v2.numpy())
    assert not np.array_equal(v1.numpy(), v3.numpy())
    assert abs(float((v1.abs() ** 2).mean()) - 2.0) < 0.5
