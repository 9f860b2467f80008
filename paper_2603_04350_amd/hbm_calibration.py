"""Plain device-to-device copy of known size, run under rocprofv3 --pmc to
calibrate what FETCH_SIZE / WRITE_SIZE report per byte actually moved.

    python -m paper_2603_04350_amd.hbm_calibration [MiB] [repeats]

Each copy reads and writes `MiB` MiB (default 512) with torch's copy kernel.
"""
import sys

import torch


def main():
    mib = int(sys.argv[1]) if len(sys.argv) > 1 else 512
    reps = int(sys.argv[2]) if len(sys.argv) > 2 else 5
    n = mib * (1 << 20) // 8
    x = torch.rand(n, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(f"copied {mib} MiB x {reps}", flush=True)


if __name__ == "__main__":
    main()
