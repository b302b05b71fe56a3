"""Plain device-to-device copy of a known size, used to calibrate the
FETCH_SIZE / WRITE_SIZE hardware counters against bytes actually moved."""
import sys

import torch


def main(mib=512, reps=3):
    n = mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(f"copy_calib: {reps} copies of {n * 4} bytes (read {n * 4} B, write {n * 4} B each)",
          flush=True)


if __name__ == "__main__":
    main(*(int(a) for a in sys.argv[1:]))
