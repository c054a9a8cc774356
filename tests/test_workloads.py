"""The synthetic inputs: stimulus masks from integer indices, the seeded
unstructured shell (validity, size, degree, edge lengths, fibres)."""
import numpy as np
import pytest

from workloads.configs import get_config, stim_mask
from workloads.tetmesh import endo_patch_mask, min_volume, shell_mesh


def test_box_masks():
    assert stim_mask(get_config("c1_2d_hh")).sum() == 49          # 7 x 7 corner nodes
    assert stim_mask(get_config("c2_3d_crn")).sum() == 16 ** 3      # 1.5 mm cube, h = 0.1
    m = stim_mask(get_config("c5_3d_crn_large")).reshape(101, 601, 601)
    assert m[:, :, :16].all() and not m[:, :, 16:].any()


def test_small_shell_is_valid_and_deterministic():
    a = shell_mesh(5, 48, 24)
    b = shell_mesh(5, 48, 24)
    assert np.array_equal(a["coords"], b["coords"]) and np.array_equal(a["tets"], b["tets"])
    assert min_volume(a["coords"], a["tets"]) > 0
    assert a["tets"].shape[0] == 6 * 4 * 48 * 23
    f = a["fibres"]
    assert np.allclose(np.linalg.norm(f, axis=1), 1.0)


@pytest.mark.slow
def test_full_shell_size_edges_and_degree():
    m = shell_mesh()
    N = m["coords"].shape[0]
    assert abs(N - 1.0e6) <= 0.05e6
    X, T = m["coords"], m["tets"]
    assert min_volume(X, T) > 0
    e = np.concatenate([np.linalg.norm(X[T[:, a]] - X[T[:, b]], axis=1) for a, b in [(0, 1), (1, 2), (2, 3)]])
    assert e.min() >= 0.19 and np.median(e) <= 0.5
    # at most 14 neighbours per node (Kuhn split): count unique edges per node
    pairs = np.concatenate([T[:, [a, b]] for a in range(4) for b in range(4) if a != b])
    key = np.unique(pairs[:, 0] * N + pairs[:, 1])
    deg = np.bincount(key // N, minlength=N)
    assert deg.max() <= 14
    assert endo_patch_mask(m).sum() >= 20
