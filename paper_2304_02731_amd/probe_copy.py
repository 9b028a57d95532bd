"""Plain streaming kernel of known size, for scaling the HBM byte counters.

Reads and writes exactly ``--mib`` MiB each per launch (y = -x over FP64),
so that ``FETCH_SIZE`` / ``WRITE_SIZE`` of the same rocprofv3 pass can be
compared with the true traffic.  Run under
``rocprofv3 --pmc FETCH_SIZE --kernel-trace -- python3 paper_2304_02731_amd/probe_copy.py``
(and again with ``WRITE_SIZE``).
"""
from __future__ import annotations

import argparse
import json


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    import torch
    n = args.mib * (1 << 20) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(args.reps):
        torch.neg(x, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"bytes_read_per_launch": n * 8, "bytes_written_per_launch": n * 8,
                      "launches": args.reps}), flush=True)


if __name__ == "__main__":
    main()
