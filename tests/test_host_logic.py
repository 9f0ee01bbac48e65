"""Host-side logic that needs no GPU: the bench contract's GPU-count check, the
traffic-record freshness rule, and the warm-start model file round trip."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_traffic_record_used_only_on_matching_source(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "profiles")
    src = tmp_path / "paper_1904_07497_amd" / "csrc"
    os.makedirs(src)
    for f in bench.KERNEL_SOURCES["sweep"]:
        (src / f).write_text("// " + f)
    rec = {"bytes_per_launch": 123, "kernel_source_sha": bench.kernel_source_sha("sweep")}
    (tmp_path / "profiles" / "traffic_sweep_large.json").write_text(json.dumps(rec))
    assert bench.load_traffic("sweep", "large") == 123
    (src / bench.KERNEL_SOURCES["sweep"][0]).write_text("// changed")
    assert bench.load_traffic("sweep", "large") is None
    assert bench.load_traffic("sweep", "video") is None


def test_warmstart_model_round_trip(tmp_path):
    torch = pytest.importorskip("torch")
    from paper_1904_07497_amd import warmstart as ws
    p = ws.init_params(16, 4)
    path = tmp_path / "m.npz"
    ws.save_model(torch.from_numpy(p), 16, path, meta={"note": "test"})
    q, hidden, seed = ws.load_model(path, device="cpu")
    assert hidden == 16 and seed == ws.SKETCH_SEED
    assert np.array_equal(q.numpy(), p)


def test_stored_model_matches_its_width():
    torch = pytest.importorskip("torch")
    from paper_1904_07497_amd import respca as rp
    from paper_1904_07497_amd import warmstart as ws
    q, hidden, _ = ws.load_model(device="cpu")
    assert q.numel() == rp.mlp_param_count(hidden) and hidden == 256
    assert torch.isfinite(q).all()
