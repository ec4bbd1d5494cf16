"""Checkpoint round trip on the host (no GPU): arrays bit for bit, parameters and seeds."""
import numpy as np
import pytest

from paper_2004_08146_amd import checkpoint
from synth import random_links, random_spinors, seed_for


def test_checkpoint_round_trip(tmp_path):
    dims = (4, 4, 4, 4)
    U = random_links(dims, 0.5, seed_for(1, "U"))
    W = random_spinors(dims, 3, seed_for(1, "W"))
    x = random_spinors(dims, 2, seed_for(1, "x"))
    params = {"tol": 1e-10, "restart": 6, "mg_prec": "f32", "taus": [0.01, -0.02]}
    seeds = {"U": seed_for(1, "U"), "W": seed_for(1, "W")}
    p = tmp_path / "ck.npz"
    checkpoint.save(p, U, W=W, x=x, params=params, seeds=seeds)
    got = checkpoint.load(p)
    assert np.array_equal(got["U"], U) and got["U"].dtype == U.dtype
    assert np.array_equal(got["W"], W) and np.array_equal(got["x"], x)
    assert got["params"] == params and got["seeds"] == seeds


def test_checkpoint_optional_parts_and_no_pickle(tmp_path):
    dims = (4, 4, 4, 4)
    U = random_links(dims, 0.5, 3)
    p = tmp_path / "u.npz"
    checkpoint.save(p, U)
    got = checkpoint.load(p)
    assert "W" not in got and "x" not in got and got["params"] == {} and got["seeds"] == {}
    with pytest.raises(TypeError):
        checkpoint.save(tmp_path / "bad.npz", U, W=np.array([object()], dtype=object))
