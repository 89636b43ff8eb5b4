"""Reference kernel of known HBM traffic for scaling the FETCH_SIZE /
WRITE_SIZE counters: an elementwise kernel that reads 1 GiB and writes 1 GiB
(y = x + 0 over 2^28 float32), run 3 times.

Usage (under rocprofv3 --pmc ...): python -m paper_2602_12098_amd.copyref
"""
import torch

N = 1 << 28   # float32 elements: 1 GiB


def main():
    x = torch.empty(N, dtype=torch.float32, device="cuda:0")   # no fill kernel: only the adds are counted
    y = torch.empty_like(x)
    for _ in range(3):
        torch.add(x, 0.0, out=y)
    torch.cuda.synchronize()
    print(f"copyref: {3} launches, {4 * N} bytes read and written each", flush=True)


if __name__ == "__main__":
    main()
