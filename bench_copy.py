"""A plain device-to-device copy of a known size: the reference against which
the HBM byte counters (FETCH_SIZE, WRITE_SIZE) of the benchmark's kernels are
scaled.  Run it under the same counter passes as the kernel being measured:

    rocprofv3 --pmc FETCH_SIZE -d <out> -o run -- python3 bench_copy.py 1024
    rocprofv3 --pmc WRITE_SIZE -d <out> -o run -- python3 bench_copy.py 1024

It moves MiB mebibytes of reads and the same of writes in one copy kernel.
"""
import json
import sys


def main():
    mib = int(sys.argv[1]) if len(sys.argv) > 1 else 1024
    import torch
    n = mib << 20
    src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n}))


if __name__ == "__main__":
    main()
