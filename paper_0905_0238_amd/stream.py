"""A survey too large for one workspace, solved in pair-range batches on one GPU.

The +-k_m pairs are independent problems (paper, Section 2.1: the Born
inversion decouples per midpoint wavenumber), so a survey can be cut into
contiguous ranges of its pairs and each range planned, assembled and solved
on its own.  Every batch plan shares the survey's |k| classes, so one Green's
table (computed once per pass) serves them all; the batches run one after
another on the current stream and share one workspace and one Gram buffer,
sized for the largest batch.  The data rows of every batch stay resident.

Batches are cut from the per-pair row counts (``pair_rows``) so that each
holds at most ``batch_rows`` data rows and ``batch_pairs`` pairs; the plans of
the batches are built on host threads (the planner releases the GIL).  With
an HBM budget, the planner refuses a batch whose pass does not fit it, and the
stream refuses a layout (all batches resident) that does not.  The data rows
may be kept in complex64 (``data="c64"``), half the bytes of complex128.
"""
from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor

import numpy as np
import torch

from .edt import Plan, pair_rows

__all__ = ["cut_batches", "Stream"]


def cut_batches(rows: np.ndarray, batch_rows: int, batch_pairs: int) -> list[tuple[int, int]]:
    """Contiguous pair ranges [a, b) covering every pair, each with at most
    ``batch_pairs`` pairs and ``batch_rows`` rows (a single pair with more
    rows than that forms a batch of its own)."""
    if batch_rows < 1 or batch_pairs < 1:
        raise ValueError("batch_rows and batch_pairs must be positive")
    out = []
    a, acc = 0, 0
    for q, r in enumerate(np.asarray(rows, np.int64)):
        if q > a and (acc + r > batch_rows or q - a >= batch_pairs):
            out.append((a, q))
            a, acc = q, 0
        acc += int(r)
    if len(rows):
        out.append((a, len(rows)))
    return out


class Stream:
    """Buffers and batch plans of one survey, precision and damping; ``step``
    runs one pass over all batches: green once, then assemble -> solve per
    batch.  ``v`` (n_km x nz) receives every batch's k_m; ``x``, ``info`` and
    ``steps`` are indexed by the survey's pair order."""

    def __init__(self, survey, prec="fp16x3", lambda_rel=None, refine_tol=3e-6, max_refine=8,
                 batch_rows=100_000_000, batch_pairs=4096, chunk_rows=0, gram_band=0, device="cuda",
                 threads=8, also=(), data="c128", hbm_budget=0):
        self.s, self.prec = survey, prec
        self.lam = float(survey.lambda_rel if lambda_rel is None else lambda_rel)
        self.tol, self.maxr = float(refine_tol), int(max_refine)
        self.precs = [prec] + [q for q in also if q != prec]
        need32 = any(q != "fp64" for q in self.precs)
        self.rows = pair_rows(survey)
        self.batches = cut_batches(self.rows, batch_rows, batch_pairs)

        # every batch plan checks that one pass of it (its device plan,
        # workspace, data and buffers, with the survey's tables and V~) fits
        # the budget; the planner refuses one that does not (EDT_ENOMEM)
        def mk(r):
            return Plan(survey, chunk_rows=chunk_rows, gram_band=gram_band, device=device, pairs=r, data=data,
                        hbm_budget=hbm_budget)

        with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
            self.plans = list(ex.map(mk, self.batches))
        if hbm_budget:
            need = self.planned_bytes()
            if need > hbm_budget:
                raise MemoryError(f"the stream needs {need} device bytes, more than the budget of {hbm_budget}")
        dev = torch.device(device)
        p0 = self.plans[0]
        nz = p0.nz
        self.n_km, self.nz = p0.n_km, nz
        self.n_pairs = int(p0.n_pairs_all)
        work = max(int(p.info["work_bytes"]) for p in self.plans)
        self.work = torch.empty(max(work, 256), dtype=torch.uint8, device=dev)
        for p in self.plans:
            p.upload(work=self.work)
        pmax = max(p.n_pairs for p in self.plans)
        self.gram = torch.empty(max(pmax, 1), nz, nz, dtype=torch.float64, device=dev)
        self.rhs = torch.empty(max(pmax, 1), 2, nz, dtype=torch.float64, device=dev)
        self.trace = torch.empty(max(pmax, 1), dtype=torch.float64, device=dev)
        self.x = torch.zeros(self.n_pairs, 2, nz, dtype=torch.float64, device=dev)
        self.info = torch.zeros(self.n_pairs, dtype=torch.int32, device=dev)
        self.steps = torch.zeros(self.n_pairs, dtype=torch.int32, device=dev)
        self.v = torch.zeros(self.n_km, nz, dtype=torch.complex128, device=dev)
        self.G64 = torch.empty(*p0.table_shape, dtype=torch.complex128, device=dev)
        self.G32 = torch.empty(*p0.table_shape, dtype=torch.complex64, device=dev) if need32 else None
        self.vel = torch.as_tensor(np.asarray(survey.vel, np.float64), device=dev).contiguous().clone()
        self.d = [None] * len(self.plans)
        self.graphs = {}

    def planned_bytes(self) -> int:
        """Device bytes the stream will hold, from the plans alone: every
        batch's device plan and data rows, one workspace and one Gram buffer
        for the largest batch, the survey's tables, x, info, steps and V~."""
        ps = self.plans
        nz = ps[0].nz
        datum = 8 if ps[0].data_dtype == torch.complex64 else 16
        per_batch = sum(int(p.info["dev_plan_bytes"]) + p.n_rows * 2 * datum for p in ps)
        work = max(int(p.info["work_bytes"]) for p in ps)
        pmax = max(max(p.n_pairs for p in ps), 1)
        gram = pmax * (nz * nz + 2 * nz + 1) * 8
        n_pairs, n_km = int(ps[0].n_pairs_all), int(ps[0].n_km)
        tables = int(ps[0].info["table_elems"]) * 24
        outs = n_pairs * (2 * nz * 8 + 8) + n_km * nz * 16
        return per_batch + work + gram + tables + outs

    def set_data(self, b: int, d_rows):
        """Data rows of batch b ([rows of the batch, 2], converted to the plan's
        data type), kept resident."""
        p = self.plans[b]
        if tuple(d_rows.shape) != (p.n_rows, 2):
            raise ValueError(f"batch {b} needs ({p.n_rows}, 2) data rows")
        if p.n_rows == 0:   # a batch of empty pairs still passes a valid pointer
            d_rows = torch.zeros(1, 2, dtype=p.data_dtype)
        self.d[b] = d_rows.to(device=self.work.device, dtype=p.data_dtype).contiguous()

    def step(self, prec=None):
        """One pass in precision ``prec`` (default: the stream's first)."""
        prec = self.prec if prec is None else prec
        if prec not in self.precs:
            raise ValueError(f"precision {prec} was not declared for this stream")
        if any(d is None for d in self.d):
            raise RuntimeError("set_data for every batch first")
        mixed = prec != "fp64"
        self.plans[0].green(self.vel, want32=mixed, out=(self.G64, self.G32 if mixed else None))
        for p, d, (a, b) in zip(self.plans, self.d, self.batches):
            P = p.n_pairs
            if P == 0:
                continue
            gram, rhs, trace = self.gram[:P], self.rhs[:P], self.trace[:P]
            p.assemble(self.G64, self.G32, d, prec, out=(gram, rhs, trace))
            p.solve(self.G64, d, gram, rhs, trace, self.lam, refine=mixed, refine_tol=self.tol,
                    max_refine=self.maxr, data_summed=True,
                    out=(self.x[a:b], self.v, self.info[a:b], self.steps[a:b]))
        return self.v

    def capture(self, prec=None, warmup: int = 1):
        """Record one pass into a HIP graph (after eager warm-up passes on a side stream)."""
        prec = self.prec if prec is None else prec
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            for _ in range(warmup):
                self.step(prec)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.step(prec)
        self.graphs[prec] = g
        return g

    def replay(self, prec=None):
        prec = self.prec if prec is None else prec
        if prec not in self.graphs:
            raise RuntimeError("capture() first")
        self.graphs[prec].replay()
        return self.v

    def resident_bytes(self) -> dict:
        """Device bytes held, by kind."""
        plans = sum(int(p.info["dev_plan_bytes"]) for p in self.plans)
        data = sum(0 if d is None else d.numel() * d.element_size() for d in self.d)
        tabs = self.G64.numel() * 16 + (0 if self.G32 is None else self.G32.numel() * 8)
        bufs = sum(t.numel() * t.element_size() for t in (self.gram, self.rhs, self.trace, self.x, self.info,
                                                          self.steps, self.v))
        return {"plans": plans, "data": data, "tables": tabs, "work": self.work.numel(), "buffers": bufs}
