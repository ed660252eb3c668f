"""Input generator: determinism, shapes and the structural invariants of the
synthetic workloads (no method arithmetic is involved)."""
import numpy as np

from paper_1011_4687_amd import synth


def test_tiny_shape_and_determinism():
    env, pts = synth.workload("tiny")
    env2, pts2 = synth.workload("tiny")
    assert env.digest() == env2.digest()
    assert synth.digest(pts) == synth.digest(pts2)
    assert env.n_nuclei == 12 and env.nbf == 84 and len(env.shells) == 60
    assert pts.shape == (1024, 3)
    assert np.all(np.linalg.norm(pts, axis=1) < 4.0)
    assert np.all(np.linalg.norm(env.xyz, axis=1) >= 4.0)
    assert np.all(np.abs(env.xyz) <= 8.0)
    assert set(np.unique(env.Z)).issubset({1.0, 6.0, 7.0, 8.0})
    assert env.blocks[0].shape == (84, 84)
    for s in env.shells:
        assert len(s.exponents) == 1 and 0.1 <= s.exponents[0] <= 50.0


def test_first_points_do_not_depend_on_count():
    _, a = synth.workload("tiny", n_points=10)
    _, b = synth.workload("tiny", n_points=1000)
    assert np.array_equal(a, b[:10])


def test_mid_structure():
    env, pts = synth.workload("mid", n_points=64)
    assert env.n_nuclei == 200 and env.n_fragments == 20
    assert np.all(np.linalg.norm(env.xyz, axis=1) >= 8.0)
    assert np.all(np.abs(env.xyz) <= 20.0)
    assert np.all(np.linalg.norm(pts, axis=1) < 8.0)
    # fragments are contiguous in the atom and basis order; blocks PSD, symmetric
    assert np.all(np.diff(env.fragment) >= 0)
    for f, blk in enumerate(env.blocks):
        assert np.allclose(blk, blk.T)
        assert np.min(np.linalg.eigvalsh(blk)) > -1e-9 * np.max(np.abs(blk))
        n = env.bf_hi[f] - env.bf_lo[f]
        assert blk.shape == (n, n)
        # rank ceil(n/2)
        assert np.linalg.matrix_rank(blk) == (n + 1) // 2
    for s in env.shells:
        assert 3 <= len(s.exponents) <= 6
        assert np.all(np.diff(s.exponents) < 0)
        assert np.all((s.coefs >= 0.1) & (s.coefs <= 1.0))
        assert np.all((s.exponents >= 0.05) & (s.exponents <= 5000.0))
    heavy = env.Z > 1
    per_atom = np.bincount([s.atom for s in env.shells], minlength=200)
    assert np.all(per_atom[heavy] == 6) and np.all(per_atom[~heavy] == 3)


def test_csr_matches_dense():
    env, _ = synth.workload("tiny", n_points=1)
    rowp, col, val = env.density_csr([2.0])
    D = env.density_dense([2.0])
    R = np.zeros_like(D)
    for i in range(D.shape[0]):
        R[i, col[rowp[i]:rowp[i + 1]]] = val[rowp[i]:rowp[i + 1]]
    assert np.array_equal(R, D)


def test_batched_instances_shapes():
    inst = synth.batched_instances(n_inst=3, max_points=50)
    for env, pts in inst:
        assert env.n_nuclei % 10 == 0 and 50 <= env.n_nuclei <= 2000
        assert pts.shape[0] <= 50
