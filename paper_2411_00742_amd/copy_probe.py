"""A plain device-to-device copy of known size, used to calibrate the HBM
traffic counters (FETCH_SIZE, WRITE_SIZE) that the benchmark's roofline
reports: the counters read over this copy, divided by the bytes it must move,
give the scale factor applied to the solver kernels' readings."""
import sys

import torch

MIB = int(sys.argv[1]) if len(sys.argv) > 1 else 512


def main():
    n = MIB * (1 << 20) // 8
    a = torch.rand(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied {MIB} MiB three times ({MIB * 1024} KiB read and written per copy)")


if __name__ == "__main__":
    main()
