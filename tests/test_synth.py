"""Seeded input generator: determinism, orthonormality, workload shapes."""
import numpy as np

from synth import (batched_specs, config_spec, make_orbitals, smooth_test_vectors,
                   training_specs, box_length_for)


def test_seeded_and_bitwise_deterministic():
    a = make_orbitals(config_spec("c1"))
    b = make_orbitals(config_spec("c1"))
    assert a.psi.tobytes() == b.psi.tobytes()
    c = make_orbitals(config_spec("c1").replace(seed=1002))
    assert np.abs(a.psi - c.psi).max() > 1e-3


def test_orthonormal_on_grid_and_delocalized():
    o = make_orbitals(config_spec("c1"))
    s = o.spec
    P = o.psi.reshape(s.norb, -1)
    np.testing.assert_allclose(P @ P.T * s.dV, np.eye(s.norb), atol=1e-12)
    assert o.cond_S < 1e4
    assert o.psi.shape == (8, 24, 24, 24)


def test_config_shapes():
    for name, (norb, n) in {"c2": (128, 96), "c3": (256, 120), "c5": (512, 160)}.items():
        s = config_spec(name)
        assert (s.norb, s.N) == (norb, n)
    assert abs(box_length_for(32) - 18.62) < 0.01


def test_batched_and_training_recipes():
    b = batched_specs()
    assert len(b) == 16
    assert all(8 <= s.n_mol <= 64 and s.N in (48, 64, 80, 96) for s in b)
    assert all(s.L / s.N <= 0.25 for s in b)
    t = training_specs(20)
    assert all(32 <= s.n_mol <= 64 and s.L / s.N <= 0.196 for s in t)
    assert len({s.seed for s in t}) == 20


def test_smooth_vectors_normalized():
    s = config_spec("c1")
    x = smooth_test_vectors(s, 4)
    np.testing.assert_allclose((x.reshape(4, -1) ** 2).sum(1) * s.dV, 1.0, rtol=1e-12)


def test_md_steps_are_small_displacements():
    s0 = config_spec("c1")
    a = make_orbitals(s0)
    assert make_orbitals(s0.replace(md_step=0)).psi.tobytes() == a.psi.tobytes()
    b = make_orbitals(s0.replace(md_step=1))
    c = make_orbitals(s0.replace(md_step=2))
    n = s0.norb
    Pa, Pb, Pc = (x.psi.reshape(n, -1) for x in (a, b, c))
    np.testing.assert_allclose(Pb @ Pb.T * s0.dV, np.eye(n), atol=1e-12)
    # same mixing matrix, centres moved by 0.05 bohr per step: the occupied
    # spaces stay close and drift further with every step
    def gap(P, Q):
        return n - np.linalg.norm(P @ Q.T * s0.dV) ** 2
    assert 0 < gap(Pa, Pb) < gap(Pa, Pc) < 0.05 * n
    d = np.linalg.norm(b.gauss_centres - a.gauss_centres, axis=1)
    np.testing.assert_allclose(np.minimum(d, s0.L - d), 0.05, rtol=1e-12)
