"""A plain device copy of known size (torch's copy kernel, 256 MiB read and
256 MiB written, three times), run under rocprofv3 --pmc to scale the HBM byte
counters FETCH_SIZE and WRITE_SIZE: for this kernel each should read 262144
KiB per dispatch; the ratio measured / 262144 is the counters' scale factor.

python -m paper_0711_0999_amd.copyprobe"""
import torch


def main():
    n = 256 << 20
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {n} bytes x 3", flush=True)


if __name__ == "__main__":
    main()
