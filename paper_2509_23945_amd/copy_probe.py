"""Plain device-to-device copy of a known size (64 MiB, three times).

Run under `rocprofv3 --pmc FETCH_SIZE` and `--pmc WRITE_SIZE` to scale those
counters to bytes: the copy reads and writes exactly 64 MiB per dispatch."""
import torch


def main() -> None:
    n = 64 * 1024 * 1024 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copied", a.numel() * 8, "bytes x 3", flush=True)


if __name__ == "__main__":
    main()
