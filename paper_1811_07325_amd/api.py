"""Torch-facing convenience over the C ABI: tensors in, device pointers out.

PyTorch supplies device memory (operands, results, the workspace) and streams;
the multiply itself runs in libstark.so.
"""
from __future__ import annotations

import torch

from . import stark as S


class Stark:
    """One library context on one device.

    workspace_bytes: if given, a torch-allocated workspace of that size is lent
    to the context; otherwise the library allocates its own as needed.
    """

    def __init__(self, device: int = 0, workspace_bytes: int | None = None, hbm_budget_bytes: int = 0,
                 max_slots: int = 0, tuner_cache: str | None = None):
        self.device = torch.device("cuda", device)
        self.workspace = None
        if workspace_bytes:
            self.workspace = torch.empty(workspace_bytes, dtype=torch.uint8, device=self.device)
        self.ctx = S.stark_create(device, self.workspace, workspace_bytes or 0, hbm_budget_bytes, max_slots,
                                  tuner_cache)

    def close(self) -> None:
        if self.ctx is not None:
            S.stark_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _check(t: torch.Tensor, n: int, name: str) -> None:
        if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != (n, n):
            raise ValueError(f"{name} must be a contiguous float32 CUDA tensor of shape ({n}, {n})")

    def gemm(self, A: torch.Tensor, B: torch.Tensor, C: torch.Tensor | None = None, depth: int = S.STARK_DEPTH_AUTO,
             precision: str | int = "bf16x3", stream=None) -> torch.Tensor:
        n = A.shape[0]
        self._check(A, n, "A")
        self._check(B, n, "B")
        if C is None:
            C = torch.empty((n, n), dtype=torch.float32, device=A.device)
        self._check(C, n, "C")
        prec = S.PRECISIONS[precision] if isinstance(precision, str) else precision
        if stream is None:
            stream = torch.cuda.current_stream(A.device)
        S.stark_gemm(self.ctx, A, B, C, n, depth, prec, stream)
        return C
