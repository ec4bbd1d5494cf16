"""GPU-test fixtures: build inputs with synth, hand identical bits to the HIP path."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_08146_amd import qmg  # noqa: F401  (raises if libqmg.so is missing)
    return qmg


def case(msg):
    print("[gpu case] " + msg, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def coarse_to_lex(yc_gpu, order, ntv):
    """GPU coarse vectors [nrhs][nb(internal order)][2ntv] -> oracle order [nrhs][nb][2ntv]."""
    nb = len(order)
    y = yc_gpu.reshape(-1, nb, 2 * ntv)
    out = np.empty_like(y)
    out[:, order, :] = y
    return out


def lex_to_coarse(y_lex, order):
    return np.ascontiguousarray(y_lex[..., order, :])


_BIG = {}


def big_inputs(dims, eps, cfg, nrhs):
    """Links and spinors of a large lattice, generated once per process."""
    from synth import random_links, random_spinors, seed_for
    key = (dims, eps, cfg)
    if key not in _BIG:
        _BIG.clear()
        _BIG[key] = random_links(dims, eps, seed_for(cfg, "U"))
    return _BIG[key], random_spinors(dims, nrhs, seed_for(cfg, "b"))
