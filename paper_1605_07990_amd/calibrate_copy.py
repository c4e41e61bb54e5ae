"""Plain device-to-device copy of a known size, for scaling hardware byte
counters: run it under `rocprofv3 --pmc FETCH_SIZE` (then WRITE_SIZE) and
divide the bytes it moves by what the counter reports per dispatch."""
from __future__ import annotations

import argparse
import json


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    import torch

    n = args.mib << 20
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(args.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"bytes_read_per_copy": n, "bytes_written_per_copy": n, "copies": args.reps}), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
