"""Host-side checkpoint of a solve's inputs: gauge field, test vectors, solver and
setup parameters, seeds.  One `.npz` file, arrays only (no pickled objects): the
parameters are stored as a JSON string.  Fields are stored in the canonical layout
of the binding (`Lattice.unpack` / `Lattice.pack`), so a checkpoint does not depend
on the device layout.  A stopped solve resumes from its saved x with
`qmg_params.x0 = 1`."""
import json

import numpy as np

_FORMAT = 1


def save(path, U, W=None, x=None, params=None, seeds=None):
    """Write U (complex [T,Z,Y,X,4,3,3]), optional test vectors W and solution x
    (complex [n,T,Z,Y,X,4,3]), parameters (a dict of numbers and strings) and seeds
    (a dict of integers) to `path` (.npz)."""
    arrays = {"format": np.array(_FORMAT), "U": np.ascontiguousarray(np.asarray(U))}
    if W is not None:
        arrays["W"] = np.ascontiguousarray(np.asarray(W))
    if x is not None:
        arrays["x"] = np.ascontiguousarray(np.asarray(x))
    meta = {"params": dict(params or {}), "seeds": {k: int(v) for k, v in (seeds or {}).items()}}
    arrays["meta"] = np.array(json.dumps(meta, sort_keys=True))
    for k, v in arrays.items():
        if v.dtype == object:
            raise TypeError("checkpoint entries must be numeric arrays: %s" % k)
    np.savez(path, **arrays)


def load(path):
    """Read a checkpoint written by `save`: dict with 'U', optional 'W' and 'x',
    'params' and 'seeds'."""
    with np.load(path, allow_pickle=False) as z:
        if int(z["format"]) != _FORMAT:
            raise ValueError("unknown checkpoint format %d" % int(z["format"]))
        out = {k: z[k] for k in ("U", "W", "x") if k in z.files}
        meta = json.loads(str(z["meta"]))
    out["params"] = meta["params"]
    out["seeds"] = meta["seeds"]
    return out
