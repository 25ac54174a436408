"""Host-side pieces of bench.py (no GPU): the dominant kernel's algorithmic
byte count, the gating of the measured-traffic figure on the kernel source
it was taken on, and the refusal of more than one GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_algorithmic_bytes_of_the_keyframe_kernel():
    # per factor: keyframe-side Jacobian, s and message (16 floats),
    # landmark-side Jacobian, its J a and message (13), the linearised
    # residual (2), landmark index, counter and flags; both messages and the
    # counter written: 171 B; per keyframe its slot, 27 + 6 doubles in and
    # 27 out; per landmark 9 doubles
    assert bench.FACTOR_BYTES_PER_FACTOR == 171
    kf = lambda nf, nk, nl, due=0: bench.step_bytes(nf, nk, nl, due, 0, 0, False)["k_factor_kf"]  # noqa: E731
    assert kf(1, 0, 0) == 171
    assert kf(0, 1, 0) == 496
    assert kf(0, 0, 1) == 72
    assert kf(10, 0, 0, due=1) == 9 * 171 + 70


def test_step_bytes_of_the_other_launches():
    """Each launch's per-unit figure, one unit at a time."""
    sb = lambda *a: bench.step_bytes(*a)  # noqa: E731
    # relinearisation: 316 B per due factor, every keyframe's belief and
    # anchor once, the landmarks it touches once
    assert sb(1, 0, 0, 0, 0, 0, False)["k_relin"] == 0
    assert sb(1, 1, 1, 1, 0, 0, False)["k_relin"] == 316 + 264 + 96
    # landmark beliefs: 56 B per edge, 104 B per landmark, 636 B per keyframe
    assert sb(1, 0, 0, 0, 0, 0, False)["k_belief_lm"] == 56
    assert sb(0, 1, 1, 0, 0, 0, False)["k_belief_lm"] == 636 + 104
    # residuals and check: 26 B per factor (35 B with a reference in FP32),
    # 36 B per checked factor, 16 B per queued factor, 144 / 48 B per
    # keyframe / landmark, 140 B per residual block
    assert sb(1, 0, 0, 0, 0, 0, False)["k_reproj_block"] == 26
    assert sb(1, 0, 0, 0, 0, 0, True)["k_reproj_block"] == 35
    assert sb(1, 0, 0, 0, 1, 0, False)["k_reproj_block"] == 26 + 36
    assert sb(0, 1, 1, 0, 0, 1, False)["k_reproj_block"] == 144 + 48 + 140


def _profile(tmp_path, sha, nbytes="577144814"):
    d = tmp_path / "profiles"
    d.mkdir(exist_ok=True)
    (d / "traffic_k_factor_kf_w.txt").write_text(
        "# HBM traffic\nhbm_bytes_per_launch: %s\nkernel_sha: %s\n" % (nbytes, sha))


def test_traffic_is_reported_only_for_the_kernel_source_it_was_taken_on(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_sha", lambda: "0123456789abcdef")
    assert bench.measured_traffic("w") is None            # no profile
    _profile(tmp_path, "0123456789abcdef")
    assert bench.measured_traffic("w") == 577144814
    _profile(tmp_path, "fedcba9876543210")               # taken on other source
    assert bench.measured_traffic("w") is None
    _profile(tmp_path, "0123456789abcdef", "n/a")        # unreadable figure
    assert bench.measured_traffic("w") is None


def test_kernel_sha_covers_the_kernel_sources():
    sha = bench.kernel_sha()
    assert len(sha) == 16 and int(sha, 16) >= 0


def test_code_only_drops_comments_and_keeps_code():
    src = "int a = 1;  // one\n/* block\n   comment */\n\nint b = a / 2; /* inline */ int c;\n"
    assert bench.code_only(src) == "int a = 1;\nint b = a / 2;  int c;"
    # a change of comments only leaves the code, a change of code does not
    assert bench.code_only(src.replace("one", "the first")) == bench.code_only(src)
    assert bench.code_only(src.replace("a / 2", "a / 3")) != bench.code_only(src)


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), ([], {"WORLD_SIZE": "2"})])
def test_more_than_one_gpu_is_refused(argv, env):
    e = dict(os.environ, **env)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv], env=e,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
