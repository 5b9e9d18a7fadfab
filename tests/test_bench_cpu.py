"""Host logic of bench.py on the CPU: the one-GPU contract, the rule that
counter-measured traffic is reported only while the kernel's sources are the
ones it was measured on, and the algorithmic byte counts per unit of work
that the roofline and the per-kernel GB/s divide by (the figures stated for
each kernel: 1652 B per active row for Adam, 56 B per instance plus 20 B per
pixel for the forward compositing, and so on)."""
import hashlib
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def _hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2605_20150_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def test_traffic_only_while_the_sources_are_unchanged(monkeypatch):
    src = ["raster_bwd.hip", "raster.h"]
    monkeypatch.setattr(bench, "TRAFFIC", {"render_bwd": {"bytes": 123.0, "sources": src,
                                                          "sha256_16": _hash(src)}})
    assert bench.measured_traffic("render_bwd") == 123.0
    assert bench.measured_traffic("render_fwd") is None
    monkeypatch.setattr(bench, "TRAFFIC", {"render_bwd": {"bytes": 123.0, "sources": src,
                                                          "sha256_16": "0" * 16}})
    assert bench.measured_traffic("render_bwd") is None


def test_executed_instructions_only_while_the_sources_are_unchanged(monkeypatch):
    src = ["raster_bwd.hip", "raster.h"]
    entry = {"valu_wave_instr": 5.0e8, "cycles_per_valu_per_simd": 3.5, "sources": src}
    monkeypatch.setattr(bench, "ISSUE", {"render_bwd": dict(entry, sha256_16=_hash(src))})
    got = bench.measured_issue("render_bwd")
    assert got["valu_wave_instr_per_launch"] == 5.0e8 and got["cycles_per_valu_per_simd"] == 3.5
    assert bench.measured_issue("render_fwd") is None
    monkeypatch.setattr(bench, "ISSUE", {"render_bwd": dict(entry, sha256_16="0" * 16)})
    assert bench.measured_issue("render_bwd") is None


def test_committed_traffic_entry_names_existing_sources():
    for kernel, t in bench.TRAFFIC.items():
        assert kernel in bench.KERNELS
        assert t["bytes"] > 0 and len(t["sha256_16"]) == 16
        for f in t["sources"]:
            assert os.path.exists(os.path.join(ROOT, "paper_2605_20150_amd", "csrc", f))


def test_algorithmic_bytes_per_unit():
    ab = bench.algorithmic_bytes
    zero = dict(n_pidx=0, n_kept=0, n_vis=0, n_inst=0, n_active=0, pixels=0, V=4)

    def one(kernel, **kw):
        args = dict(zero)
        args.update(kw)
        return ab(kernel, args["n_pidx"], args["n_kept"], args["n_vis"], args["n_inst"], args["n_active"],
                  args["pixels"], args["V"])

    assert one("adam", n_active=1) == 7 * 236 == 1652
    assert one("render_fwd", n_inst=1) == 56 and one("render_fwd", pixels=1) == 20
    assert one("render_bwd", n_inst=1) == 92 and one("render_bwd", pixels=1) == 20
    assert one("reduce_pairs", n_vis=1) == 48 and one("reduce_pairs", n_inst=1) == 36
    assert one("adjoint", n_active=1) == 480 and one("adjoint", n_vis=1) == 36
    # the fused stage saves the gradient's write and read and the second read
    # of the parameters (3 x 236 per active row) and counts the step
    # counter's read and write, which the adam figure leaves out
    assert one("adjoint_adam", n_active=1) == one("adjoint", n_active=1) + one("adam", n_active=1) - 3 * 236 + 8
    assert one("adjoint_adam", n_vis=1) == 36
    assert one("loss_fwd", pixels=1) == 3 * 20 and one("loss_bwd", pixels=1) == 3 * 24
    # preprocess: 16 B per pidx plus 4 B of cull output per invisible pair,
    # 224 B per kept Gaussian, 64 B per visible pair
    assert one("preprocess", n_pidx=1, V=1) == 16 + 4
    assert one("preprocess", n_kept=1) == 224
    assert one("preprocess", n_pidx=1, n_vis=1, V=1) == 16 + 64
    assert one("emit", n_inst=10) == 0   # not a bandwidth figure


def test_cpu_model_names_the_sockets():
    assert "socket" in bench.cpu_model()


def test_compositing_work_per_visit_is_the_stated_model():
    """The ALU roofline counts the method's per-visit formulas: about 20
    operations and one exponential per forward visit, about 50 and two
    transcendentals per backward visit."""
    assert bench.FLOPS_PER_FWD_VISIT == 21
    assert bench.FLOPS_PER_BWD_VISIT == 52
    assert set(bench.HBM_BOUND) <= set(bench.KERNELS + bench.UNFUSED)
    assert "render_bwd" not in bench.HBM_BOUND and "render_fwd" not in bench.HBM_BOUND
