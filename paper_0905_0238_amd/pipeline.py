"""One full pass of the hot path on preallocated buffers, and its capture
into a HIP graph.

A pass is green -> assemble -> solve (paper, Section 2.1: the reference
Green's tables, the per-pair damped normal equations of eqs. DMV / Split and
their solution, recombined by eq. VSym).  Every buffer is allocated once here;
a pass only launches library kernels on the current stream, which makes it
capturable: the library issues no allocation, copy or memset on this path and
the refinement loop has a fixed launch count (pairs that have converged exit
at once).
"""
from __future__ import annotations

import torch

__all__ = ["Pipeline"]


class Pipeline:
    """Buffers for one plan, precision and damping; ``step`` runs one pass.

    prec: "fp64" (FP64 Gram, no refinement) or "bf16x3" / "fp32" (mixed Gram
    with FP64 refinement to ``refine_tol``, at most ``max_refine`` steps).
    """

    def __init__(self, plan, vel, d_rows, lambda_rel, prec="fp64", refine_tol=1e-6, max_refine=8):
        dev = plan.device
        self.p, self.prec, self.lam = plan, prec, float(lambda_rel)
        self.tol, self.maxr = float(refine_tol), int(max_refine)
        self.mixed = prec != "fp64"
        P, nz = plan.n_pairs, plan.nz
        plan.upload()
        self.vel = vel.to(device=dev, dtype=torch.float64).contiguous().clone()
        self.d = d_rows.to(device=dev, dtype=plan.data_dtype).contiguous().clone()
        self.G64 = torch.empty(*plan.table_shape, dtype=torch.complex128, device=dev)
        self.G32 = torch.empty(*plan.table_shape, dtype=torch.complex64, device=dev) if self.mixed else None
        self.gram = torch.zeros(P, nz, nz, dtype=torch.float64, device=dev)
        self.rhs = torch.empty(P, 2, nz, dtype=torch.float64, device=dev)
        self.trace = torch.empty(P, dtype=torch.float64, device=dev)
        self.x = torch.empty(P, 2, nz, dtype=torch.float64, device=dev)
        self.v = torch.empty(plan.n_km, nz, dtype=torch.complex128, device=dev)
        self.info = torch.empty(P, dtype=torch.int32, device=dev)
        self.steps = torch.zeros(P, dtype=torch.int32, device=dev)
        self.graph = None

    def set_data(self, d_rows):
        """Copy new data rows in place (the captured graph reads this buffer)."""
        self.d.copy_(d_rows)

    def step(self):
        p = self.p
        p.green(self.vel, want32=self.mixed, out=(self.G64, self.G32))
        p.assemble(self.G64, self.G32, self.d, self.prec, out=(self.gram, self.rhs, self.trace))
        p.solve(self.G64, self.d, self.gram, self.rhs, self.trace, self.lam, refine=self.mixed,
                refine_tol=self.tol, max_refine=self.maxr, data_summed=True,
                out=(self.x, self.v, self.info, self.steps))
        return self.v

    def capture(self, warmup: int = 1):
        """Record one pass into a HIP graph (after `warmup` eager passes on a
        side stream, as graph capture requires)."""
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            for _ in range(warmup):
                self.step()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.step()
        self.graph = g
        return g

    def replay(self):
        if self.graph is None:
            raise RuntimeError("capture() first")
        self.graph.replay()
        return self.v
