"""bench.py's contract on the host: more than one GPU is refused with a JSON
message before anything touches a GPU; the algorithmic byte counts per
matrix are the inputs read once and the outputs written once; the counter
and accuracy summaries are used only while their recorded source digest
matches the kernel sources."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_algorithmic_bytes():
    f64, f32 = 8, 4
    assert bench.BYTES["fwd_general_f64"] == (9 + 3) * f64
    assert bench.BYTES["fwd_symmetric_f64"] == (6 + 3) * f64
    assert bench.BYTES["fwd_symmetric_f32"] == (6 + 3) * f32
    assert bench.BYTES["fwd_general_f32"] == (9 + 3) * f32
    assert bench.BYTES["bwd_general_f64"] == (9 + 3 + 9) * f64
    assert bench.BYTES["step_general_f64"] == bench.BYTES["fwd_general_f64"] + bench.BYTES["bwd_general_f64"]
    assert bench.BYTES["eigenprojectors_general_f64"] == (9 + 27) * f64
    assert bench.BYTES["matrix_function_backward_general_f64"] == (9 + 9 + 9) * f64


def test_summaries_follow_the_source_digest(tmp_path, monkeypatch):
    digest = bench.source_digest()
    assert len(digest) == 64
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    if rec.get("source_sha256") == digest:
        assert bench.traffic_record("bwd_general_f64_fma") is not None
    # a summary taken on other sources is not used
    fake = tmp_path / "profiles"
    fake.mkdir()
    (fake / "traffic.json").write_text(json.dumps({**rec, "source_sha256": "0" * 64}))
    (fake / "accuracy.json").write_text(json.dumps({"source_sha256": "0" * 64, "rows": []}))
    monkeypatch.setattr(bench, "source_digest", lambda: digest)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_record("bwd_general_f64_fma") is None
    assert bench.accuracy_report() is None
    assert bench.stated_accuracy(None) is None
    assert bench.within_8x(None, "differentiation batch, general f64", "double_word") is None


def test_stated_accuracy_from_a_report():
    out = {"gpu_vs_exact": {"max": 2.5, "p9999": 1.5}, "gpu_vs_O1": {"max": 40.0, "p9999": 9.0},
           "O1_vs_exact": {"max": 41.0, "p9999": 9.5}, "g12_fail": 0, "t8_fail": 0, "elements": 10}
    bad = {**out, "t8_fail": 3}
    rep = {"rows": [{"workload": "w", "mode": "double_word", "n": 10, "outputs": {"eigvals": out, "J3": out}},
                    {"workload": "w", "mode": "fma", "n": 10, "outputs": {"eigvals": bad, "J3": out}}],
           "adjoint": {"double_word": {"gpu": 1e-11, "paper_route": 5e-11}}}
    s = bench.stated_accuracy(rep)
    assert s["w"]["double_word"]["within_8x_bound"] is True
    assert s["w"]["fma"]["within_8x_bound"] is False
    assert s["w"]["double_word"]["eigvals"]["vs_exact_p9999"] == 1.5
    assert bench.within_8x(rep, "w", "double_word") is True
    assert bench.within_8x(rep, "w", "fma") is False
    assert bench.within_8x(rep, "other", "fma") is None
