"""A plain device copy of known size (512 MiB read, 512 MiB written, three
times), whose FETCH_SIZE / WRITE_SIZE counter readings scale the counters of
the GEMM kernel to bytes."""
import torch

n = 64 * 1024 * 1024  # doubles: 512 MiB
a = torch.ones(n, dtype=torch.float64, device="cuda")
b = torch.empty_like(a)
for _ in range(3):
    b.copy_(a)
torch.cuda.synchronize()
print("copied", n * 8, "bytes x3", flush=True)
