"""Host-side behaviour of bench.py that needs no GPU: a request for more than
one GPU is refused with a message and exit status 2 before anything touches
a device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and p.stdout == ""


def _bench():
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import bench
    return bench


def test_every_hbm_roofline_gets_the_attainable_bandwidth():
    bench = _bench()
    rec = {"roofline": {"bound": "hbm", "achieved": 24.0},
           "residual": {"roofline_mixed": {"bound": "hbm", "achieved": 3000.0},
                        "roofline_fp64": {"bound": "mfma", "achieved": 32.0}},
           "secondary": {"a": {"roofline": {"bound": "alu", "achieved": 0.2}},
                         "b": {"c": {"roofline": {"bound": "hbm", "achieved": 6.0}}}}}
    bench.add_attainable(rec, 5000.0)
    assert rec["roofline"]["attainable"] == 5000.0 and rec["roofline"]["frac_of_attainable"] == 24.0 / 5000.0
    assert rec["residual"]["roofline_mixed"]["frac_of_attainable"] == 0.6
    assert rec["secondary"]["b"]["c"]["roofline"]["attainable"] == 5000.0
    assert "attainable" not in rec["residual"]["roofline_fp64"]
    assert "attainable" not in rec["secondary"]["a"]["roofline"]


def test_blocked_error_of_a_k_by_l_cur_matches_the_direct_one():
    import numpy as np
    import torch
    bench = _bench()
    g = torch.Generator().manual_seed(3)
    A = torch.randn(2500, 300, generator=g)
    I = torch.randint(0, 2500, (24,), generator=g)
    J = torch.randint(0, 300, (17,), generator=g)
    U = torch.randn(17, 24, generator=g, dtype=torch.float64)
    W = A.double()
    ref = float(torch.linalg.norm(W - W[:, J] @ U @ W[I]) / torch.linalg.norm(W))
    assert np.isclose(bench.rel_err_k_by_l(torch, A, I, J, U, rows=700), ref, rtol=1e-12)


def test_counter_table_entries_name_existing_sources():
    bench = _bench()
    for line, (src, sha, fetch, write, cf, cw) in bench.TRAFFIC_COUNTS.items():
        assert all(os.path.exists(os.path.join(ROOT, f)) for f in src), line
        assert len(sha) == 40 and fetch > 0 and write > 0 and cf > 0 and cw > 0
