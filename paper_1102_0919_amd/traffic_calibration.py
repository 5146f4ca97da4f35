"""Plain device copy of a known size, run under rocprofv3 --pmc to calibrate the HBM byte counters.

    rocprofv3 --pmc FETCH_SIZE -d DIR -o NAME -- python3 -m paper_1102_0919_amd.traffic_calibration

The copy reads and writes exactly COPY_BYTES each (float64 tensors, far larger than the caches), so
FETCH_SIZE and WRITE_SIZE per dispatch of the copy kernel divided by COPY_BYTES give the factor that
turns the counters of other kernels into bytes.
"""
from __future__ import annotations

import sys

COPY_BYTES = 1 << 30     # 1 GiB read + 1 GiB written per copy
REPEATS = 3


def main() -> int:
    import torch
    if not torch.cuda.is_available():
        print("traffic_calibration: needs a HIP device", file=sys.stderr)
        return 2
    n = COPY_BYTES // 8
    src = torch.empty(n, dtype=torch.float64, device="cuda").uniform_()
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(REPEATS):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {COPY_BYTES} bytes {REPEATS} times", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
