"""The GPU invariant checker (lopc_verify) against the tests' own CPU
restatement of the definitions (tests/topo.py): error bound, edge orders and
critical types, on round trips (no violation) and on planted changes."""
import numpy as np
import pytest
import torch

from paper_2603_26968_amd import synth
import topo

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_26968_amd as P
    return P


def cpu_report(x, y, eps):
    d = np.abs(x.astype(np.float64) - y.astype(np.float64))  # exact for float32
    eo = topo.edge_orders(x)
    ey = topo.edge_orders(y)
    tx = topo.critical_points(x)
    ty = topo.critical_points(y)
    return {"points": x.size, "max_abs_error": float(d.max()),
            "edges": int(sum(e.size for e in eo)),
            "order_violations": int(sum((a != b).sum() for a, b in zip(eo, ey))),
            "types_orig": [int((tx == t).sum()) for t in range(4)],
            "types_recon": [int((ty == t).sum()) for t in range(4)],
            "type_mismatches": int((tx != ty).sum())}


CASES = [
    ("bumps2d", lambda: synth.gaussian_bumps((70, 61), seed=2), 1e-3),
    ("bumps3d", lambda: synth.gaussian_bumps((14, 12, 17), seed=4, sigma_range=(2, 8)), 1e-2),
    ("noise3d_f64", lambda: np.random.default_rng(3).standard_normal((9, 10, 11)), 1e-1),
    ("plane3d", lambda: np.random.default_rng(4).standard_normal((1, 20, 30)).astype(np.float32), 1e-2),
    ("point", lambda: np.array([[0.5]], np.float32), 1e-3),
]


@pytest.mark.parametrize("name,make,eb", CASES, ids=[c[0] for c in CASES])
def test_round_trip_keeps_every_invariant(P, ref, name, make, eb):
    print("[case] verify", name, flush=True)
    x = make()
    s = ref.compress(x, eb, ref.NOA if x.size > 1 else ref.ABS)
    y = ref.decompress(s)
    eps = ref.stream_info(s)["eps"]
    rep = P.verify(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda(), eps)
    want = cpu_report(x, y, eps)
    for k, v in want.items():
        assert rep[k] == v, (name, k, rep[k], v)
    assert rep["bound_violations"] == 0 and rep["order_violations"] == 0
    assert rep["type_mismatches"] == 0


def test_planted_changes_are_counted(P, ref):
    print("[case] verify planted", flush=True)
    x = synth.gaussian_bumps((40, 52), seed=3)
    s = ref.compress(x, 1e-3, ref.NOA)
    y = ref.decompress(s).copy()
    eps = ref.stream_info(s)["eps"]
    y[5, 7], y[5, 8] = y[5, 8], y[5, 7]              # may swap an edge order
    y[20, 30] = np.float32(y[20, 30] + 3 * eps)      # out of bound
    y[33, 10] = np.float32(x.max() + 1.0)            # a new maximum
    rep = P.verify(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda(), eps)
    want = cpu_report(x, y, eps)
    for k, v in want.items():
        assert rep[k] == v, (k, rep[k], v)
    d = np.abs(x.astype(np.float64) - y.astype(np.float64))
    assert rep["bound_violations"] == int((d > eps).sum()) >= 2
    assert rep["order_violations"] > 0 and rep["type_mismatches"] > 0


def test_full_size_round_trip(P):
    """turb3d 256^3 through the GPU path: no invariant broken."""
    print("[case] verify turb3d 256^3", flush=True)
    x = torch.from_numpy(synth.turbulence_field()).cuda()
    s, st = P.compress(x, 1e-3, "noa", stats=True)
    y = P.decompress(s)
    rep = P.verify(x, y, st["eps"])
    assert rep["points"] == x.numel()
    assert rep["bound_violations"] == 0 and rep["order_violations"] == 0
    assert rep["type_mismatches"] == 0 and rep["max_abs_error"] <= st["eps"]
    # one edge per positive offset d in {0,1}^3 \ 0 and every p with p + d in the grid
    assert rep["edges"] == sum((256 - a) * (256 - b) * (256 - c)
                               for a in (0, 1) for b in (0, 1) for c in (0, 1) if a or b or c)
