"""Local coherence lc(v) = ||Pi v|| / ||v|| (Sec. 3.1) on the GPU: parity with the
oracle, and a synthetic reproduction of the paper's 4^4 local-coherence study for Q."""
import numpy as np
import pytest

from gpu_common import case, dev, host, need_gpu
from oracle import clover as oclover
from oracle import dense, mg
from synth import random_links, random_spinors, seed_for

pytestmark = pytest.mark.gpu

DIMS, BLOCK = (4, 4, 4, 4), (2, 2, 2, 2)


def _lat(csw=1.0, m0=-0.5):
    qmg = need_gpu()
    U = random_links(DIMS, 0.5, seed_for(11, "U"))
    lat = qmg.Lattice(DIMS, BLOCK)
    lat.set_gauge(dev(U), m0, csw)
    return qmg, lat, U


def test_local_coherence_matches_oracle():
    case("local coherence 4^4 parity")
    qmg, lat, U = _lat()
    W = random_spinors(DIMS, 24, seed_for(11, "W"))
    lat.set_test_vectors(lat.pack(dev(W)), 24)
    P = mg.build_P(W, BLOCK)
    V = np.concatenate([random_spinors(DIMS, 40, 7), W], axis=0)
    got = lat.local_coherence(lat.pack(dev(V)), len(V))
    ref = np.array([mg.local_coherence(P, v, BLOCK) for v in V])
    assert np.max(np.abs(got - ref)) < 1e-12
    assert np.allclose(got[40:], 1.0, atol=1e-12)


def test_local_coherence_study_Q():
    """The paper's experiment for Q on 4^4 with synthetic links: the full spectrum
    in natural order, interpolation sets of 24 consecutive eigenvectors (every
    4th of the 128 sets here), P from each set with 2^4 aggregates, lc of all
    3072 eigenvectors.  Checked: lc = 1 inside the set; coherence well above
    the no-coherence level sqrt(768/3072) = 0.5 for the eigenvectors of
    smallest |lambda| when P comes from the central set; and higher next to the
    set than far from it."""
    case("local coherence study 4^4 Q")
    qmg, lat, U = _lat()
    C = oclover.clover_term(U, 1.0)
    w, v = np.linalg.eigh(dense.dense_Q(U, -0.5, C))        # ascending = natural real order
    N = len(w)
    X = v.T.reshape((N,) + DIMS + (4, 3))
    Xg = lat.pack(dev(X))
    fb = lat.field_bytes()
    nsets = N // 24
    center = int(np.argmin(np.abs(w)))
    center_set = center // 24
    sets = sorted(set(list(range(0, nsets, 4)) + [center_set]))
    small = np.argsort(np.abs(w))[:N // 10]                 # the 10% smallest |lambda|
    summary = {}
    for sidx in sets:
        lo = 24 * sidx
        lat.set_test_vectors(Xg[lo * fb:(lo + 24) * fb], 24)
        lc = np.concatenate([lat.local_coherence(Xg[k * fb:(k + 64) * fb], 64) for k in range(0, N, 64)])
        assert np.allclose(lc[lo:lo + 24], 1.0, atol=1e-10)
        near = np.r_[max(0, lo - 48):lo, lo + 24:min(N, lo + 72)]
        far = np.r_[0:48, N - 48:N] if 48 <= lo < N - 72 else np.arange(N // 2 - 24, N // 2 + 24)
        summary[sidx] = (float(np.mean(lc[near])), float(np.mean(lc[far])),
                         float(np.mean(np.delete(lc[small], np.isin(small, np.arange(lo, lo + 24))))))
    print("[lc] set: (mean lc next to the set, far from it, over the 10% smallest |lambda|)")
    for k in sorted(summary):
        print("[lc] %3d %s" % (k, tuple(round(x, 3) for x in summary[k])))
    c_near, c_far, c_small = summary[center_set]
    assert c_small > 0.6, summary[center_set]
    assert c_near > c_far, summary[center_set]
    assert np.mean([summary[k][0] for k in summary]) > 0.5
