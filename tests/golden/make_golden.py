"""Writes the golden streams in this folder.  It calls only the oracle.

The inputs are exact dyadic rationals built from integer formulas, so they
are bit-identical on every machine.  The streams freeze this project's
container layout (the paper does not describe a byte layout, so the layout
itself is pinned only by these fixtures and by round trips); the values they
encode are pinned by the oracle's own tests.

Run:  python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402


def golden_inputs():
    """name -> (array, eb, mode).  Values are integers / 64 (exact)."""
    out = {}
    i, j = np.meshgrid(np.arange(23), np.arange(31), indexing="ij")
    v = ((i * 37 + j * 101 + (i * j) % 7) % 29 - 14) / 64.0
    out["grid2d_f32_noa"] = (v.astype(np.float32), 0.05, oracle.NOA)
    out["grid2d_f64_abs"] = (v.astype(np.float64), 0.125, oracle.ABS)
    a, b, c = np.meshgrid(np.arange(6), np.arange(5), np.arange(7), indexing="ij")
    w = ((a * 13 + b * 7 + c * 3 + (a * b * c) % 5) % 17 - 8) / 32.0
    out["grid3d_f32_abs"] = (w.astype(np.float32), 0.2, oracle.ABS)
    out["grid3d_f64_noa"] = (w.astype(np.float64), 0.1, oracle.NOA)
    # a chain falling with the index inside one bin (worst case of Sec. IV-E)
    out["chain_f32"] = (np.linspace(0.75, 0.25, 65).astype(np.float32).reshape(1, 65), 1.0, oracle.ABS)
    # more than one chunk (4096 float32 points per chunk), ragged last chunk
    k = np.arange(70 * 61)
    x = (((k * 2654435761) % 1021) - 510) / 256.0
    out["two_chunks_f32"] = (x.reshape(70, 61).astype(np.float32), 0.01, oracle.NOA)
    return out


def main():
    oracle.build(force=False)
    index = {}
    for name, (x, eb, mode) in golden_inputs().items():
        s = oracle.compress(x, eb, mode)
        with open(os.path.join(HERE, name + ".hex"), "w") as f:
            hx = s.hex()
            for p in range(0, len(hx), 96):
                f.write(hx[p:p + 96] + "\n")
        index[name] = {"shape": list(x.shape), "dtype": str(x.dtype), "eb": eb,
                       "mode": "NOA" if mode == oracle.NOA else "ABS", "bytes": len(s)}
    with open(os.path.join(HERE, "index.json"), "w") as f:
        json.dump(index, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main()
