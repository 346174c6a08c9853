"""CPU checks of bench.py's host logic: the one-GPU guard and the rule that a
recorded traffic figure is reported only for the kernel source it was
measured on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_recorded_traffic_only_for_measured_source(monkeypatch):
    digest = bench.bcr_source_digest()
    assert len(digest) == 64
    rec = dict(kernel_src_sha256=digest, bytes_per_launch=123, fetch_bytes_per_launch=100,
               write_bytes_per_launch=23, summary="x")
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", rec)
    assert bench.recorded_traffic("k_bcr") == 123
    assert bench.recorded_traffic("k_gemm") is None
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", dict(rec, kernel_src_sha256="0" * 64))
    assert bench.recorded_traffic("k_bcr") is None
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", None)
    assert bench.recorded_traffic("k_bcr") is None


def test_recorded_summary_exists():
    rec = bench.TRAFFIC_RECORD
    if rec:
        assert os.path.exists(os.path.join(ROOT, rec["summary"]))
        assert rec["bytes_per_launch"] == rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]


@pytest.mark.parametrize("argv", [[], ["--steps", "5", "--warmup", "2"]])
def test_default_solve_options(argv):
    a = bench.parse(argv)
    assert a.gpus == 1 and a.config == "C2"
    o = bench.solve_options(a)
    assert o["inner_mode"] in (1, 2) and o["precision"] == 0


def test_traffic_digest_follows_the_pass_kernels_and_the_factorization(tmp_path, monkeypatch):
    # the recorded traffic stays valid exactly while the pass kernels and the
    # host factorization are unchanged
    import shutil
    src = os.path.join(ROOT, "paper_1906_06785_amd", "csrc")
    dst = tmp_path / "paper_1906_06785_amd" / "csrc"
    dst.mkdir(parents=True)
    for f in ("kernels.hip", "host_setup.cpp", "solver.hip"):
        shutil.copy(os.path.join(src, f), dst / f)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    d0 = bench.bcr_source_digest()

    def edit(name, anchor, extra):
        p = dst / name
        text = p.read_text()
        i = text.index(anchor)
        p.write_text(text[:i] + extra + text[i:])

    # outside both sections: same digest
    edit("kernels.hip", "// ------------------------------------------------------------------ truncation", "// note\n")
    edit("host_setup.cpp", "void bcr_factor(", "// note\n")
    assert bench.bcr_source_digest() == d0
    # inside the pass kernels
    edit("kernels.hip", "constexpr int BCR_MAXBS", "// note\n")
    d1 = bench.bcr_source_digest()
    assert d1 != d0
    # inside the factorization
    edit("host_setup.cpp", "  constexpr int NT = BcrFactor::NT, NTOP", "  // note\n")
    d2 = bench.bcr_source_digest()
    assert d2 != d1
    # the launch side: variant table, grid padding and tuning
    edit("kernels.hip", "  const unsigned gx = 8 * cdiv(no, 8);", "  // note\n")
    d3 = bench.bcr_source_digest()
    assert d3 != d2
    edit("kernels.hip", "std::vector<int> bcr_tune(", "// note\n")
    d4 = bench.bcr_source_digest()
    assert d4 != d3
    # the device layout of a factor
    edit("solver.hip", "    const int mode = f.pass_mode[p];", "    // note\n")
    d5 = bench.bcr_source_digest()
    assert d5 != d4
    # the rest of solver.hip does not count
    edit("solver.hip", "// ====================================================================== C ABI", "// note\n")
    assert bench.bcr_source_digest() == d5
    # the time loop that lays out the passes' right-hand sides counts; the
    # graph capture around it does not
    edit("solver.hip", "  const long blk = (long)S.nu * nxi;\n  if (f32) {", "  // note\n")
    d6 = bench.bcr_source_digest()
    assert d6 != d5
    edit("solver.hip", "bool mean_loop_graph(", "// note\n")
    assert bench.bcr_source_digest() == d6
