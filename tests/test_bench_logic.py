"""Host-side checks of the bench's accounting (no GPU needed): the algorithmic
byte count of the forward pass, and the HBM traffic read from committed
rocprofv3 counters, which must be withheld once the kernel source differs
from the one the counters were taken on."""
import hashlib
import json
import os

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2601_08552_amd", "csrc", "lecqmc_kernels.hip")


def test_algorithmic_bytes_of_the_forward_pass():
    # 32x32 dilute gas: N = 1024, 8 + 8, 320 slices, a QR every 10 slices.
    # Per spin and slice Phi_R and Phi_L in and out (4 N Ne 8 bytes), per
    # block and spin 5 N Ne 8 bytes, plus a read and a write byte per field.
    N, ne, L, nb = 1024, 8, 320, 32
    want = 2 * (L * 4 * N * ne * 8 + nb * 5 * N * ne * 8) + 2 * L * N
    assert bench.algorithmic_bytes_forward(N, ne, ne, L, 10) == want
    # a ragged last block counts as a block; an empty spin adds nothing
    assert bench.algorithmic_bytes_forward(16, 2, 0, 45, 10) == 45 * 4 * 16 * 2 * 8 + 5 * 5 * 16 * 2 * 8 + 2 * 45 * 16


def _record(tmp_path, sha):
    rec = {"src_sha256": sha, "fetch_kib_per_dispatch": 1000.0, "write_kib_per_dispatch": 300.0,
           "fetch_scale": 2.0, "write_scale": 1.0}
    p = tmp_path / "pmc.json"
    p.write_text(json.dumps(rec))
    return str(p)


def test_traffic_from_counters_of_the_same_source(tmp_path):
    sha = hashlib.sha256(open(SRC, "rb").read()).hexdigest()
    got = bench.measured_traffic(SRC, _record(tmp_path, sha))
    assert got == (1000.0 * 2.0 + 300.0 * 1.0) * 1024.0


def test_traffic_withheld_after_a_source_change(tmp_path):
    assert bench.measured_traffic(SRC, _record(tmp_path, "0" * 64)) is None
    assert bench.measured_traffic(SRC, str(tmp_path / "missing.json")) is None


def test_committed_counter_record_is_well_formed():
    rec = json.load(open(os.path.join(ROOT, "profiles", "k_forward_batched256_pmc.json")))
    for k in ("kernel", "workload", "src_file", "src_sha256", "fetch_kib_per_dispatch", "write_kib_per_dispatch",
              "fetch_scale", "write_scale", "calibration"):
        assert k in rec, k
    assert len(rec["src_sha256"]) == 64 and rec["fetch_kib_per_dispatch"] > 0 and rec["write_kib_per_dispatch"] > 0


def test_more_than_one_gpu_is_refused_before_any_device_work():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]
