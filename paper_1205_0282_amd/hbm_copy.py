"""Reference for HBM traffic counters: a plain device-to-device copy of a known
number of bytes (1 GiB by default), repeated.  Run under a counter collection
(FETCH_SIZE / WRITE_SIZE); the counters reported for the copy kernel divided
by the bytes it moved give the scale applied to the ray caster's counters.

    python -m paper_1205_0282_amd.hbm_copy [--mib 1024] [--reps 3]
"""
import argparse

import torch


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--mib", type=int, default=1024)
    p.add_argument("--reps", type=int, default=3)
    a = p.parse_args()
    n = a.mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(a.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {a.mib} MiB x {a.reps}: read {n * 4} B and wrote {n * 4} B per copy", flush=True)


if __name__ == "__main__":
    main()
