"""Plain device-to-device copy of a known size, for calibrating HBM counters.

    python -m paper_2002_11401_amd.membench --mib 1024 --reps 5

Copies a `mib`-MiB buffer `reps` times with PyTorch's copy kernel and prints
the achieved bandwidth (read + write bytes / time).  Under
`rocprofv3 --pmc FETCH_SIZE` (then WRITE_SIZE) the counters of one copy
dispatch, divided by the bytes the copy must move, give the scale factor
that turns the counter readings of the full-field pass into bytes.
"""
from __future__ import annotations

import argparse
import json
import time


def main():
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args()
    n = a.mib * (1 << 20)
    src = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / a.reps
    print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n,
                      "seconds_per_copy": dt, "GBps_read_plus_write": 2 * n / dt / 1e9}))


if __name__ == "__main__":
    main()
