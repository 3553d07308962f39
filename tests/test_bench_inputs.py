"""The benchmark evaluates the large inputs of the paper's Neumann examples on
the device; on the CPU its generators must give synth's arrays (same
definitions: Section 6.2 eq. ex2d1, Section 6.3 eq. ex3d1, the degree-4
polynomial perturbation)."""

import numpy as np
import pytest

import synth

bench = pytest.importorskip("bench")


@pytest.mark.parametrize("n", [5, 9, 16])
def test_device_generators_match_synth(n):
    u, f = bench.e4_inputs(n, device="cpu")
    u2, f2 = synth.neumann_2d(n)
    np.testing.assert_allclose(u.numpy(), u2, rtol=0, atol=1e-15)
    np.testing.assert_allclose(f.numpy(), f2, rtol=1e-15, atol=1e-13)
    u, f, v = bench.e7_inputs(n, device="cpu")
    u2, f2, v2 = synth.neumann_potential_3d(n)
    np.testing.assert_allclose(u.numpy(), u2, rtol=0, atol=1e-15)
    np.testing.assert_allclose(v.numpy(), v2, rtol=1e-15, atol=1e-13)
    np.testing.assert_allclose(f.numpy(), f2, rtol=1e-14, atol=1e-12)
    for dim in (2, 3):
        for seed in (0, 3):
            np.testing.assert_allclose(bench.perturbation(n, dim, seed, device="cpu").numpy(),
                                       synth.polynomial_perturbation(n, dim, seed),
                                       rtol=0, atol=1e-14)


@pytest.mark.parametrize("n", [5, 12])
def test_eigen_inputs_match_synth(n):
    v, u = bench.e8_inputs(n, device="cpu")
    v2, u2 = synth.schrodinger_3d(n)
    np.testing.assert_allclose(v.numpy(), v2, rtol=1e-15, atol=1e-12)
    np.testing.assert_allclose(u.numpy(), u2, rtol=1e-15, atol=1e-300)
    c = synth.interior_coords(n, -8.0, 8.0)
    np.testing.assert_allclose(bench.perturbation(n, 3, 2, device="cpu", coords=c).numpy(),
                               synth.polynomial_perturbation(n, 3, 2, coords=c),
                               rtol=0, atol=1e-14)
