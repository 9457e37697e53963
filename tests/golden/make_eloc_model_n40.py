"""Writes ``eloc_model_n40.json``: FP64 oracle local energies (Eq. 4 summed
over every connected configuration, amplitudes from the FP64 network of
Section 3.1) for all 32 samples of the reduced transformer workload
N=40 (K=20 spatial orbitals, 7 up + 7 down electrons), the full-E_loc recipe
at a size the oracle finishes in minutes.  Calls only ``oracle`` and the
seeded input generators; run from the repository root:

    python tests/golden/make_eloc_model_n40.py
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

RECIPE = dict(cfg=3, K=20, n_up=7, n_dn=7, n_unique=32)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "eloc_model_n40.json")


def inputs():
    kw = dict(RECIPE)
    return synth.config_inputs(kw.pop("cfg"), **kw)


def input_digest(d) -> str:
    """Digest of every input the values depend on (guards against generator drift)."""
    h = hashlib.sha256()
    for a in (d["h"], d["g"], d["keys"], d["counts"]):
        h.update(np.ascontiguousarray(a).tobytes())
    for name in sorted(d["weights"]):
        h.update(name.encode())
        h.update(np.ascontiguousarray(d["weights"][name]).tobytes())
    return h.hexdigest()[:16]


def main():
    d = inputs()
    t = time.time()
    e, ab = oracle.eloc_model(d["K"], d["n_up"], d["n_dn"], d["h"], d["g"], d["e_core"], d["weights"],
                              d["model_shape"], d["keys"], with_absum=True)
    en = oracle.energy(d["counts"], e)
    out = {
        "description": "FP64 oracle full local energies (every connected x', FP64 transformer and phase MLP) "
                       "for all samples of the reduced N=40 full-E_loc workload",
        "citation": "Eq. 4 (local energy), Eq. 6 (weighted energy over unique samples), Section 3.1 (ansatz)",
        "recipe": RECIPE, "input_sha256_16": input_digest(d),
        "connections_per_sample": oracle.n_connections(d["K"], d["n_up"], d["n_dn"]),
        "eloc_re": e.real.tolist(), "eloc_im": e.imag.tolist(), "absum": ab.tolist(),
        "energy": [float(v) for v in en], "oracle_seconds": time.time() - t,
    }
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {OUT} in {out['oracle_seconds']:.1f} s")


if __name__ == "__main__":
    main()
