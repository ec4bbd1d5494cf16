"""qmg_field_dot_noalloc (no device allocation, fixed library scratch) against
qmg_field_dot, called through the C ABI: two calls in a row, the second on a
smaller input, bitwise equal results; requests beyond the scratch are rejected."""
import ctypes

import numpy as np
import pytest

from gpu_common import case, dev, need_gpu, torch
from synth import random_spinors

pytestmark = pytest.mark.gpu


def _dots(qmg, lat, a, b, nrhs, prec, fn):
    res = (ctypes.c_double * (2 * nrhs))()
    st = getattr(qmg._lib, fn)(lat._h, res, ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), nrhs,
                               qmg._PREC[prec], ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, qmg._lib.qmg_last_error(lat._h)
    return np.array(res[:])


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_field_dot_noalloc_matches_field_dot(prec):
    case("no-alloc field dot " + prec)
    qmg = need_gpu()
    for dims, nrhs in (((16, 8, 8, 8), 16), ((8, 8, 8, 4), 3)):   # second call: a smaller input
        lat = qmg.Lattice(dims, (4, 4, 4, 4))
        a = lat.pack(dev(random_spinors(dims, nrhs, 5)), prec)
        b = lat.pack(dev(random_spinors(dims, nrhs, 6)), prec)
        ref = _dots(qmg, lat, a, b, nrhs, prec, "qmg_field_dot")
        got = _dots(qmg, lat, a, b, nrhs, prec, "qmg_field_dot_noalloc")
        assert np.array_equal(got, ref), (dims, nrhs)
        # and the values are the dot products themselves
        ca = lat.unpack(a, nrhs, prec).reshape(nrhs, -1)
        cb = lat.unpack(b, nrhs, prec).reshape(nrhs, -1)
        exact = torch.sum(torch.conj(ca) * cb, dim=1).cpu().numpy()
        assert np.allclose(got[0::2] + 1j * got[1::2], exact, rtol=1e-12, atol=0)


def test_field_dot_noalloc_rejects_oversize():
    case("no-alloc field dot: size limit")
    qmg = need_gpu()
    lat = qmg.Lattice((64, 64, 64, 32), (4, 4, 4, 4))   # 8.4M sites: 64 rhs exceed the scratch
    dummy = torch.zeros(16, dtype=torch.uint8, device="cuda")
    res = (ctypes.c_double * 128)()
    st = qmg._lib.qmg_field_dot_noalloc(lat._h, res, ctypes.c_void_p(dummy.data_ptr()),
                                        ctypes.c_void_p(dummy.data_ptr()), 64, 0,
                                        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == -1
    assert b"scratch" in qmg._lib.qmg_last_error(lat._h)
