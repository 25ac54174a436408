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
    # landmark-side Jacobian and message (11), factor-private data (10),
    # landmark index, counter and flags; both messages and the counter
    # written: 195 B; per keyframe 27 doubles in and 27 out; per landmark
    # 9 doubles
    assert bench.FACTOR_BYTES_PER_FACTOR == 195
    assert bench.factor_launch_bytes(1, 0, 0) == 195
    assert bench.factor_launch_bytes(0, 1, 0) == 432
    assert bench.factor_launch_bytes(0, 0, 1) == 72
    assert bench.factor_launch_bytes(2151544, 17940, 269085) == 446675280


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


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), ([], {"WORLD_SIZE": "2"})])
def test_more_than_one_gpu_is_refused(argv, env):
    e = dict(os.environ, **env)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv], env=e,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
