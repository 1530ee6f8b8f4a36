"""Plain device copy of a known size, for calibrating HBM traffic counters.

Run under ``rocprofv3 --pmc FETCH_SIZE`` (then ``WRITE_SIZE``) to learn what the
counters read for a copy that moves exactly ``--mib`` MiB each way; the ratio
scales the counter readings of other kernels to bytes.
"""
import argparse

import torch


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=3)
    a = ap.parse_args()
    n = a.mib * (1 << 20) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(a.reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(f"copied {a.mib} MiB x {a.reps}")


if __name__ == "__main__":
    main()
