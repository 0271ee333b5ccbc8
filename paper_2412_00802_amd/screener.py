"""The learned screener: a bf16 MLP over hashed subtree features that ranks
refinement candidates by predicted F1 (a project extension, not in the paper).

Layers: 4096 -> 1024 -> 256 -> 2 with ReLU.  The two outputs are either
logits of covered fractions (of the examples, or of a parent's coverage),
trained with BCE-with-logits, or log(1 + positives/negatives a refinement
removes from its parent), trained with the squared error; AdamW on fp32
master weights.  Every product, activation, loss, gradient and
optimiser update runs in the library's kernels (hth_gemm_bf16 on MFMA and
friends); this module only sequences the calls and owns the device buffers.
"""
from __future__ import annotations

from typing import Dict, Optional, Sequence

import numpy as np

from . import hthedl

D_IN, D_H1, D_H2, D_OUT = 4096, 1024, 256, 2


def init_params(seed: int = 7) -> Dict[str, np.ndarray]:
    """He-uniform weights and zero biases (float32), drawn on the host so that
    the same initial state can be handed to any reference."""
    rng = np.random.default_rng(seed)

    def he(fan_in, fan_out):
        lim = np.sqrt(6.0 / fan_in)
        return rng.uniform(-lim, lim, size=(fan_in, fan_out)).astype(np.float32)

    return {"w1": he(D_IN, D_H1), "b1": np.zeros(D_H1, np.float32),
            "w2": he(D_H1, D_H2), "b2": np.zeros(D_H2, np.float32),
            "w3": he(D_H2, D_OUT) * 0.5, "b3": np.zeros(D_OUT, np.float32)}


class Screener:
    """Device-resident MLP with its optimiser state and per-batch buffers."""

    def __init__(self, params: Dict[str, np.ndarray], batch: int = 1024, device: str = "cuda",
                 lr: float = 1e-3, weight_decay: float = 1e-4, loss: str = "bce"):
        """loss: "bce" (targets are fractions, BCE-with-logits) or "mse"
        (real targets, squared error)."""
        import torch
        self.t = torch
        self.loss_kind = {"bce": 0, "mse": 1}[loss]
        self.dev = torch.device(device)
        self.batch = batch
        self.lr, self.wd = lr, weight_decay
        self.b1, self.b2, self.eps = 0.9, 0.999, 1e-8
        self.step_no = 0
        f32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(self.dev)  # noqa: E731
        self.p = {k: f32(v) for k, v in params.items()}
        self.m = {k: torch.zeros_like(v) for k, v in self.p.items()}
        self.v = {k: torch.zeros_like(v) for k, v in self.p.items()}
        self.g = {k: torch.zeros_like(v) for k, v in self.p.items()}
        bf = torch.bfloat16
        self.w1b = torch.empty((D_IN, D_H1), dtype=bf, device=self.dev)
        self.w2b = torch.empty((D_H1, D_H2), dtype=bf, device=self.dev)
        # the forward products read the weights as [N][K] (both operands
        # contiguous along K); kept in step with w1b / w2b
        self.w1t = torch.empty((D_H1, D_IN), dtype=bf, device=self.dev)
        self.w2t = torch.empty((D_H2, D_H1), dtype=bf, device=self.dev)
        hthedl.hth_to_bf16(self.p["w1"], self.w1b, D_IN * D_H1)
        hthedl.hth_to_bf16(self.p["w2"], self.w2b, D_H1 * D_H2)
        self._transpose()
        B = batch
        self.x = torch.empty((B, D_IN), dtype=bf, device=self.dev)
        self.h1 = torch.empty((B, D_H1), dtype=bf, device=self.dev)
        self.h2 = torch.empty((B, D_H2), dtype=bf, device=self.dev)
        self.z = torch.empty((B, D_OUT), dtype=torch.float32, device=self.dev)
        self.dz = torch.empty((B, D_OUT), dtype=torch.float32, device=self.dev)
        self.dh2 = torch.empty((B, D_H2), dtype=bf, device=self.dev)
        self.dh1 = torch.empty((B, D_H1), dtype=bf, device=self.dev)
        self.loss = torch.zeros(1, dtype=torch.float32, device=self.dev)

    def _transpose(self) -> None:
        hthedl.hth_transpose_bf16(self.w1b, D_IN, D_H1, self.w1t)
        hthedl.hth_transpose_bf16(self.w2b, D_H1, D_H2, self.w2t)

    # -- layers -------------------------------------------------------------

    def forward(self, n: int, x=None):
        """h1, h2, z for the first n rows of self.x (or of x)."""
        x = self.x if x is None else x
        G = hthedl.hth_gemm_bf16
        G(0, 1, n, D_H1, D_IN, x, D_IN, self.w1t, D_IN, bias=self.p["b1"], relu=1, cbf=self.h1, ldcb=D_H1)
        G(0, 1, n, D_H2, D_H1, self.h1, D_H1, self.w2t, D_H1, bias=self.p["b2"], relu=1, cbf=self.h2,
          ldcb=D_H2)

    def train_step(self, n: int, y, x=None) -> None:
        """One AdamW step on rows [0, n) of x (default self.x) with targets y
        (device float32 [n][2]).  The summed loss accumulates in self.loss."""
        x = self.x if x is None else x
        G = hthedl.hth_gemm_bf16
        self.forward(n, x)
        hthedl.hth_head_forward(self.h2, n, D_H2, self.p["w3"], self.p["b3"], self.z, y, self.dz,
                                1.0 / (2 * n), self.loss, loss_kind=self.loss_kind)
        hthedl.hth_head_backward(self.h2, n, D_H2, self.p["w3"], self.dz, self.g["w3"], self.dh2)
        hthedl.hth_colsum(self.dz, 0, n, D_OUT, self.g["b3"])
        G(1, 0, D_H1, D_H2, n, self.h1, D_H1, self.dh2, D_H2, c32=self.g["w2"], ldc=D_H2)
        hthedl.hth_colsum(self.dh2, 1, n, D_H2, self.g["b2"])
        G(0, 1, n, D_H1, D_H2, self.dh2, D_H2, self.w2b, D_H2, mask=self.h1, ldm=D_H1, cbf=self.dh1,
          ldcb=D_H1)
        hthedl.hth_colsum(self.dh1, 1, n, D_H1, self.g["b1"])
        G(1, 0, D_IN, D_H1, n, x, D_IN, self.dh1, D_H1, c32=self.g["w1"], ldc=D_H1)
        self.step_no += 1
        for k in ("w1", "b1", "w2", "b2", "w3", "b3"):
            pbf = self.w1b if k == "w1" else (self.w2b if k == "w2" else None)
            hthedl.hth_adamw(self.p[k], self.g[k], self.m[k], self.v[k], pbf, self.p[k].numel(),
                             self.lr, self.b1, self.b2, self.eps, self.wd if k[0] == "w" else 0.0,
                             self.step_no)
        self._transpose()

    def logits(self, n: int, x=None):
        self.forward(n, x)
        hthedl.hth_head_forward(self.h2, n, D_H2, self.p["w3"], self.p["b3"], self.z)
        return self.z[:n]

    def params_numpy(self) -> Dict[str, np.ndarray]:
        return {k: v.detach().cpu().numpy() for k, v in self.p.items()}


class FeatureBatch:
    """Hashed features of a set of encoded hypotheses, resident on the device."""

    def __init__(self, nodes: np.ndarray, offsets: np.ndarray, children: np.ndarray, device="cuda"):
        import torch
        t = torch
        self.n_hyps = int(offsets.shape[0] - 1)
        n_nodes = int(nodes.shape[0])
        self.nodes = t.from_numpy(nodes.view(np.uint8).copy()).to(device)
        self.offsets = t.from_numpy(offsets.astype(np.int32)).to(device)
        self.children = t.from_numpy(children.astype(np.int32) if children.size else np.zeros(1, np.int32)).to(device)
        self.hash = t.empty(max(1, n_nodes), dtype=t.int64, device=device)
        self.feat = t.empty(max(1, n_nodes), dtype=t.int16, device=device)
        self.bad = t.zeros(1, dtype=t.int32, device=device)
        self.n_children = int(children.size)
        self.recompute()

    def recompute(self) -> None:
        """Hash the resident node arrays again (the features step of screening)."""
        hthedl.hth_features(self.nodes, self.offsets, self.n_hyps, self.children, self.n_children,
                            self.hash, self.feat, self.bad)

    def densify(self, row0: int, n: int, x, parents: "FeatureBatch" = None, parent_index=None,
                context: int = 0) -> None:
        """Rows [row0, row0 + n) into x; with parents (and a device uint32
        parent_index per hypothesis), minus each parent's features, and with
        context the parent's own features in the other half of the index."""
        if parents is None:
            hthedl.hth_densify(self.feat, self.offsets, row0, n, x)
        else:
            hthedl.hth_densify_delta(self.feat, self.offsets, row0, n, parents.feat, parents.offsets,
                                     parent_index, x, parent_context=context)
