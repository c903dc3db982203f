"""Reference copy for HBM traffic counters: copies a buffer of known size on
the device a few times, so that the FETCH_SIZE / WRITE_SIZE counters of a
profiler run can be scaled by what they read for exactly `bytes` read and
`bytes` written per dispatch.

    python hbm_calib.py --bytes 1073741824 --reps 3
"""
from __future__ import annotations

import argparse


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--bytes", type=int, default=1 << 30)
    ap.add_argument("--reps", type=int, default=3)
    a = ap.parse_args(argv)
    import torch
    n = a.bytes // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(a.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {a.reps} x {n * 4} bytes", flush=True)


if __name__ == "__main__":
    main()
