"""Copy probe: a device copy of a known byte count, used to scale the HBM
byte counters of a profiler run (FETCH_SIZE and WRITE_SIZE read for this
copy against the bytes it must move).  Run under the profiler as
``python -m paper_1208_0277_amd.copy_probe [MiB] [repeats]``."""

import sys


def main():
    import torch
    mib = int(sys.argv[1]) if len(sys.argv) > 1 else 1024
    reps = int(sys.argv[2]) if len(sys.argv) > 2 else 5
    n = mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.int32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(f"copy probe: {reps} copies of {mib} MiB (each reads {mib} MiB and writes {mib} MiB)", flush=True)


if __name__ == "__main__":
    main()
