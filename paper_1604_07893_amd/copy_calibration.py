"""A device copy of known size, for scaling HBM traffic counters.

    python -m paper_1604_07893_amd.copy_calibration

Copies a 64 Mi-element FP64 tensor (512 MiB) three times with torch's copy
kernel: each copy reads and writes exactly 512 MiB, so the ratio of those bytes
to what `rocprofv3 --pmc FETCH_SIZE` (or `WRITE_SIZE`) reports for one copy is
the factor that turns the counter into bytes for other kernels.
"""

import torch


def main():
    a = torch.empty(64 << 20, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copied", a.numel() * 8, "bytes x3", flush=True)


if __name__ == "__main__":
    main()
