"""Helpers shared by the GPU tests: host <-> device word tensors, LWE cases."""
import numpy as np

import oracle
import workload


def to_dev_u32(a: np.ndarray, device="cuda"):
    import torch
    a = np.ascontiguousarray(np.asarray(a, dtype=np.uint32))
    return torch.from_numpy(a.view(np.int32)).to(device)


def to_host_u32(t) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint32)


def to_dev_u8(a: np.ndarray, device="cuda"):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device)


def sample_rows(R: int, k: int, seed: int) -> np.ndarray:
    g = np.random.default_rng(seed)
    pick = g.choice(R, size=min(k, R), replace=False)
    return np.unique(np.concatenate([pick, [0, R - 1]])).astype(np.int64)


def lwe_queries(A: np.ndarray, draws: "workload.LweDraws") -> np.ndarray:
    """C x B matrix whose column b is the oracle's LWE query for draw b."""
    B = draws.s.shape[0]
    cols = [oracle.lwe_query(A, draws.s[b], draws.e[b], int(draws.col[b])) for b in range(B)]
    return np.stack(cols, axis=1)


def banner(msg: str) -> None:
    """Name the case on stdout before a GPU step (flushed)."""
    print(f"\n[gpu-case] {msg}", flush=True)
