"""A plain device copy of known size, for calibrating rocprofv3's byte
counters: three copies of exactly 1 GiB (2^27 doubles) between two device
buffers.  The counters' FETCH_SIZE / WRITE_SIZE for these dispatches divided
by 1 GiB are the scale factors applied to the kernels' counter readings.

    rocprofv3 --pmc FETCH_SIZE -- python -m paper_1810_04033_amd.calib
"""
import torch


def main():
    torch.cuda.set_device(0)
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    c = torch.empty_like(a)
    for _ in range(3):
        c.copy_(a)
    torch.cuda.synchronize()
    print("copied 3 x 1 GiB", flush=True)


if __name__ == "__main__":
    main()
