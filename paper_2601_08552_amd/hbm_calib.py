"""Plain device-to-device copy of a known size, used to calibrate the HBM
byte counters (FETCH_SIZE / WRITE_SIZE) read by rocprofv3 against the
algorithmic bytes of the sweep kernels.

    python3 -m paper_2601_08552_amd.hbm_calib [--mib 1024] [--reps 3]
"""
import argparse

import torch


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=3)
    a = ap.parse_args()
    n = a.mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(a.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {a.reps} x {a.mib} MiB", flush=True)


if __name__ == "__main__":
    main()
