"""Python face of libedt: a Plan owns the host plan, its device copy and the
workspace; every method marshals torch tensors into one C-ABI call on the
current HIP stream.  No arithmetic of the method happens here."""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib

__all__ = ["Plan", "solve", "pair_rows"]


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _structs(survey):
    """(edt_survey, edt_layers, arrays they point into) of a survey object."""
    freq = np.ascontiguousarray(survey.freqs, dtype=np.float64)
    vel = np.ascontiguousarray(survey.vel, dtype=np.float64)
    zif = np.ascontiguousarray(survey.zif, dtype=np.float64)
    dp = C.POINTER(C.c_double)
    sv = _lib.Survey(int(survey.dim), int(survey.n_mid), float(survey.d_mid),
                     int(getattr(survey, "n_off", 0)), float(getattr(survey, "d_off", 0.0)),
                     int(freq.shape[0]), freq.ctypes.data_as(dp), float(survey.eps),
                     int(survey.nz), float(survey.z0), float(survey.dz), float(survey.kappa),
                     int(getattr(survey, "n_line", 0)), float(getattr(survey, "d_line", 0.0)))
    ly = _lib.Layers(int(vel.shape[0]), vel.ctypes.data_as(dp), zif.ctypes.data_as(dp) if zif.size else None)
    return sv, ly, (freq, vel, zif)


def pair_rows(survey) -> np.ndarray:
    """Data rows of every pair of the survey (survey pair order), no plan built."""
    L = _lib.load()
    sv, ly, keep = _structs(survey)
    n = C.c_int64(0)
    i64p = C.POINTER(C.c_int64)
    _lib.check(L.edt_survey_pair_rows(C.byref(sv), C.byref(ly), C.byref(n), None), "edt_survey_pair_rows")
    out = np.zeros(n.value, np.int64)
    _lib.check(L.edt_survey_pair_rows(C.byref(sv), C.byref(ly), C.byref(n), out.ctypes.data_as(i64p)),
               "edt_survey_pair_rows")
    del keep
    return out


class Plan:
    """Rows, classes and work items of one survey, resident on one GPU.

    ``survey`` needs: dim, n_mid, d_mid, n_off, d_off, freqs, eps, nz, z0, dz,
    kappa, vel (layer velocities; vel[0] fixes c_top for the evanescent cut)
    and zif (interface depths).  ``pairs = (begin, end)`` plans only that
    range of the survey's pairs (a batch); its Green's table is the survey's.
    ``chunk_rows``, ``gram_band`` and ``resid_group`` shape the work items (0 =
    the planner's default; see paper_0905_0238_amd.tune), ``data`` is the
    storage of the data rows ("c128" or "c64") and ``hbm_budget`` (bytes, 0 =
    none) makes the planner refuse a plan whose pass would not fit.
    """

    def __init__(self, survey, chunk_rows: int = 0, gram_band: int = 0, device: str = "cuda",
                 pairs: tuple[int, int] | None = None, data: str = "c128", hbm_budget: int = 0,
                 resid_group: int = 0):
        L = _lib.load()
        self.device = torch.device(device)
        sv, ly, self._keep = _structs(survey)
        h = C.c_void_p()
        pb, pe = (0, 0) if pairs is None else (int(pairs[0]), int(pairs[1]))
        if data not in _lib.DATA_TYPES:
            raise ValueError(f"data must be one of {sorted(_lib.DATA_TYPES)}")
        opts = _lib.PlanOpts(int(chunk_rows), int(gram_band), pb, pe, _lib.DATA_TYPES[data], int(hbm_budget),
                             int(resid_group))
        _lib.check(L.edt_plan_create(C.byref(sv), C.byref(ly), C.byref(opts), C.byref(h)),
                   "edt_plan_create")
        self._h = h
        info = _lib.PlanInfo()
        _lib.check(L.edt_plan_query(h, C.byref(info)), "edt_plan_query")
        self.info = {k: getattr(info, k) for k, _ in _lib.PlanInfo._fields_}
        self.nz = int(survey.nz)
        self.dim = int(getattr(survey, "dim", 2))
        self.n_mid = int(survey.n_mid)
        self.n_line = int(getattr(survey, "n_line", 0))
        self.n_freq = int(info.n_freq)
        self.n_km = int(info.n_km)
        self.n_pairs = int(info.n_pairs)
        self.n_pairs_all = int(info.n_pairs_all)
        self.pair_begin = int(info.pair_begin)
        self.n_rows = int(info.n_rows)
        self.n_layers = int(info.n_layers)
        self.table_shape = (int(info.n_freq), int(info.n_cls), int(info.nz))
        self.data_dtype = torch.complex64 if data == "c64" else torch.complex128
        self._dev_plan = None
        self._work = None

    def _rows(self, d, what="d_rows"):
        """Check that d is a contiguous [n_rows, 2] tensor of the plan's data
        type on its device (the kernels index it by the plan's rows)."""
        shape_ok = tuple(d.shape) == (self.n_rows, 2) or (self.n_rows == 0 and d.numel() > 0)
        if (d.dtype != self.data_dtype or not shape_ok or not d.is_contiguous()
                or d.device.type != self.device.type):
            raise ValueError(f"{what} must be a contiguous ({self.n_rows}, 2) {self.data_dtype} tensor on "
                             f"{self.device}, got {tuple(d.shape)} {d.dtype} on {d.device}")
        return d

    # ----------------------------------------------------------- host side --
    def rowmap(self):
        """Host copies: row_off, rows (f, cls_r, cls_s), keys, pair_km, cls_k."""
        L = _lib.load()
        P, R = self.n_pairs, self.n_rows
        row_off = np.zeros(P + 1, np.int64)
        rows = np.zeros((R, 3), np.int32)
        keys = np.zeros((R, 2), np.int32)
        pair_km = np.zeros((P, 2), np.int32)
        cls_k = np.zeros(self.table_shape[1], np.float64)
        i64p, ip, dp = C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_double)
        _lib.check(L.edt_plan_rowmap(self._h, row_off.ctypes.data_as(i64p), rows.ctypes.data_as(ip),
                                     keys.ctypes.data_as(ip), pair_km.ctypes.data_as(ip),
                                     cls_k.ctypes.data_as(dp)), "edt_plan_rowmap")
        return dict(row_off=row_off, rows=rows, keys=keys, pair_km=pair_km, cls_k=cls_k)

    def urows(self):
        """Host copies: urow_off, urows (f, mult, cls_r, cls_s), row_unique."""
        L = _lib.load()
        U = int(self.info["n_urows"])
        urow_off = np.zeros(self.n_pairs + 1, np.int64)
        urows = np.zeros((U, 4), np.int32)
        row_unique = np.zeros(self.n_rows, np.int32)
        i64p, ip = C.POINTER(C.c_int64), C.POINTER(C.c_int32)
        _lib.check(L.edt_plan_urows(self._h, urow_off.ctypes.data_as(i64p), urows.ctypes.data_as(ip),
                                    row_unique.ctypes.data_as(ip)), "edt_plan_urows")
        return dict(urow_off=urow_off, urows=urows, row_unique=row_unique)

    def schedule(self, which: str = "gram"):
        """Host copies of the work items (pair, begin, end) and launch order."""
        L = _lib.load()
        w = {"gram": 0, "resid": 1}[which]
        i64p, ip = C.POINTER(C.c_int64), C.POINTER(C.c_int32)
        counts = np.zeros(2, np.int64)
        _lib.check(L.edt_plan_schedule(self._h, w, counts.ctypes.data_as(i64p), None, None), "edt_plan_schedule")
        items = np.zeros((int(counts[0]), 3), np.int32)
        sched = np.zeros(int(counts[1]), np.int32)
        _lib.check(L.edt_plan_schedule(self._h, w, counts.ctypes.data_as(i64p), items.ctypes.data_as(ip),
                                       sched.ctypes.data_as(ip)), "edt_plan_schedule")
        return items, sched

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().edt_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------- device side --
    def upload(self, work=None):
        """Copy the plan to the GPU and allocate the workspace (once).  ``work``
        (a uint8 tensor of at least work_bytes) is used instead of a new one:
        plans that run one after another on a stream can share it."""
        if self._dev_plan is None:
            L = _lib.load()
            nb = int(self.info["dev_plan_bytes"])
            self._dev_plan = torch.empty(max(nb, 256), dtype=torch.uint8, device=self.device)
            _lib.check(L.edt_plan_upload(self._h, _ptr(self._dev_plan), nb, _stream()), "edt_plan_upload")
        if work is not None:
            if (work.dtype != torch.uint8 or work.numel() < int(self.info["work_bytes"])
                    or work.device.type != self.device.type):
                raise ValueError("shared workspace too small or on another device")
            self._work = work
        elif self._work is None:
            self._work = torch.empty(max(int(self.info["work_bytes"]), 256), dtype=torch.uint8,
                                     device=self.device)
        return self

    def _c128(self, *shape):
        return torch.empty(*shape, dtype=torch.complex128, device=self.device)

    def _data_rows(self):
        return torch.empty(self.n_rows, 2, dtype=self.data_dtype, device=self.device)

    def green(self, vel, want32: bool = True, out=None):
        """(g64, g32) tables of shape (n_freq, n_cls, nz)."""
        self.upload()
        vel = vel.to(device=self.device, dtype=torch.float64).contiguous()
        g64 = out[0] if out else self._c128(*self.table_shape)
        g32 = (out[1] if out else torch.empty(*self.table_shape, dtype=torch.complex64,
                                              device=self.device)) if want32 else None
        _lib.check(_lib.load().edt_green(self._h, _ptr(vel), _ptr(g64), _ptr(g32), _stream()), "edt_green")
        return g64, g32

    def assemble(self, g64, g32, d_rows, prec="fp64", out=None):
        """(gram[P, nz, nz] lower triangle, rhs[P, 2, nz], trace[P])."""
        self.upload()
        P, nz = self.n_pairs, self.nz
        if out is None:
            gram = torch.zeros(P, nz, nz, dtype=torch.float64, device=self.device)
            rhs = torch.empty(P, 2, nz, dtype=torch.float64, device=self.device)
            trace = torch.empty(P, dtype=torch.float64, device=self.device)
        else:
            gram, rhs, trace = out
        self._rows(d_rows)
        _lib.check(_lib.load().edt_assemble(self._h, _ptr(g64), _ptr(g32), _ptr(d_rows),
                                            _lib.PRECISIONS[prec], _ptr(gram), _ptr(rhs), _ptr(trace),
                                            _ptr(self._work), _stream()), "edt_assemble")
        return gram, rhs, trace

    def solve(self, g64, d_rows, gram, rhs, trace, lambda_rel, refine=False, refine_tol=1e-8,
              max_refine=8, escalate=True, data_summed=False, out=None):
        """(x[P, 2, nz], v[n_km, nz] complex128, info[P], steps[P]).  With refine,
        escalate re-assembles in FP64 the pairs whose factorisation failed, and
        data_summed reuses the data sums that assemble(d_rows) left in the
        workspace (only right after that call, with d_rows unchanged)."""
        self.upload()
        P, nz = self.n_pairs, self.nz
        if out is None:
            x = torch.empty(P, 2, nz, dtype=torch.float64, device=self.device)
            v = self._c128(self.n_km, nz)
            info = torch.empty(P, dtype=torch.int32, device=self.device)
            steps = torch.zeros(P, dtype=torch.int32, device=self.device)
        else:
            x, v, info, steps = out
        if refine:
            self._rows(d_rows)
        opts = _lib.SolveOpts(1 if refine else 0, float(refine_tol), int(max_refine),
                              1 if (refine and escalate) else 0, 1 if data_summed else 0)
        _lib.check(_lib.load().edt_solve(self._h, _ptr(g64), _ptr(d_rows), _ptr(gram), _ptr(rhs), _ptr(trace),
                                         float(lambda_rel), C.byref(opts), _ptr(x), _ptr(v), _ptr(info),
                                         _ptr(steps), _ptr(self._work), _stream()), "edt_solve")
        return x, v, info, steps

    def solve_static(self, g64, d_rows, gram, rhs, trace, lambda_rel, refine=False, refine_tol=1e-8,
                     max_refine=8, escalate=True, out=None):
        """solve() through edt_solve_static: the library's static device scratch
        instead of the plan's workspace (no device allocation in the call; the
        outputs are allocated here unless ``out`` gives them)."""
        self.upload()
        P, nz = self.n_pairs, self.nz
        if out is None:
            x = torch.empty(P, 2, nz, dtype=torch.float64, device=self.device)
            v = self._c128(self.n_km, nz)
            info = torch.empty(P, dtype=torch.int32, device=self.device)
            steps = torch.zeros(P, dtype=torch.int32, device=self.device)
        else:
            x, v, info, steps = out
        if refine:
            self._rows(d_rows)
        opts = _lib.SolveOpts(1 if refine else 0, float(refine_tol), int(max_refine),
                              1 if (refine and escalate) else 0, 0)
        _lib.check(_lib.load().edt_solve_static(self._h, _ptr(g64), _ptr(d_rows), _ptr(gram), _ptr(rhs),
                                                _ptr(trace), float(lambda_rel), C.byref(opts), _ptr(x), _ptr(v),
                                                _ptr(info), _ptr(steps), _stream()), "edt_solve_static")
        return x, v, info, steps

    def tsvd(self, gram, rhs, tol_rel, max_iter=64, out=None, tsvd_work=None):
        """The paper's truncated-SVD solve from an assembled Gram (overwritten):
        (x[P, 2, nz], v[n_km, nz] complex128, info[P], iters[P]).  The default
        max_iter lets an eigenvalue of X_0 as small as about 1e-13 in magnitude
        converge: it grows 2.2 times per capped scaled step while the schedule
        scales, 1.5 times per plain step after, then quadratically (about 60
        steps); smaller ones, within rounding of the threshold, are reported as
        not converged."""
        self.upload()
        L = _lib.load()
        P, nz = self.n_pairs, self.nz
        if tsvd_work is None:
            tsvd_work = self.tsvd_work()
        if out is None:
            x = torch.empty(P, 2, nz, dtype=torch.float64, device=self.device)
            v = self._c128(self.n_km, nz)
            info = torch.empty(P, dtype=torch.int32, device=self.device)
            iters = torch.zeros(P, dtype=torch.int32, device=self.device)
        else:
            x, v, info, iters = out
        _lib.check(L.edt_tsvd(self._h, _ptr(gram), _ptr(rhs), float(tol_rel), int(max_iter), _ptr(x), _ptr(v),
                              _ptr(info), _ptr(iters), _ptr(self._work), _ptr(tsvd_work), _stream()), "edt_tsvd")
        return x, v, info, iters

    def tsvd_work(self):
        """A device workspace for tsvd and kz_restrict."""
        nb = C.c_size_t(0)
        _lib.check(_lib.load().edt_tsvd_work_bytes(self._h, C.byref(nb)), "edt_tsvd_work_bytes")
        return torch.empty(max(int(nb.value), 256), dtype=torch.uint8, device=self.device)

    def kz_disk_radius(self, factor=2.2):
        """Radius factor * 2 pi f_max / c_top of the (k_m, k_z) disk (rad/m)."""
        k = C.c_double(0.0)
        _lib.check(_lib.load().edt_kz_disk_radius(self._h, float(factor), C.byref(k)), "edt_kz_disk_radius")
        return k.value

    def kz_restrict(self, gram, rhs, k_disk, tsvd_work, n_keep=None):
        """Restrict every pair to the disk k_z^2 + |k_m|^2 <= k_disk^2 (in place on
        gram and rhs); returns n_keep[P] (int32) when asked for (n_keep=True or a
        tensor)."""
        self.upload()
        if n_keep is True:
            n_keep = torch.empty(self.n_pairs, dtype=torch.int32, device=self.device)
        _lib.check(_lib.load().edt_kz_restrict(self._h, float(k_disk), _ptr(gram), _ptr(rhs),
                                               _ptr(n_keep) if n_keep is not None else None, _ptr(tsvd_work),
                                               _stream()), "edt_kz_restrict")
        return n_keep

    def records_shape(self):
        """Shape of the shot records: (n_freq, N, N) [f, receiver, source] on the
        2D line; (n_freq, N_y, N, N) [f, line, receiver, source] for the 3D
        survey of parallel lines; (n_freq, 2N, 2N, 2N, 2N) [f, Rx, Ry, Sx, Sy]
        for the 3D areal survey (the doubled periodic survey, whose whole-grid
        wavenumbers are the rows' half-grid ones)."""
        if self.n_line:
            return (self.n_freq, self.n_line, self.n_mid, self.n_mid)
        if self.dim == 3:
            return (self.n_freq,) + (2 * self.n_mid,) * 4
        return (self.n_freq, self.n_mid, self.n_mid)

    def _check_records(self, t, what):
        want = int(np.prod(self.records_shape()))
        if t.dtype != torch.complex128 or not t.is_cuda or not t.is_contiguous() or t.numel() != want:
            raise ValueError(f"{what}: a contiguous complex128 device tensor of shape {self.records_shape()}")

    def shots_fft(self, shots):
        """In place: the shot records (records_shape(), complex128) become their
        DFT over receivers and sources, times d_mid per axis."""
        self._check_records(shots, "shots_fft")
        self.upload()
        _lib.check(_lib.load().edt_shots_fft(self._h, _ptr(shots), _stream()), "edt_shots_fft")
        return shots

    def shots_pack(self, spectrum, out=None):
        """d_rows[R, 2] (the plan's data type) of this plan's rows from a shots_fft spectrum."""
        self._check_records(spectrum, "shots_pack")
        self.upload()
        d = self._rows(out) if out is not None else self._data_rows()
        _lib.check(_lib.load().edt_shots_pack(self._h, _ptr(spectrum), _ptr(d), _stream()), "edt_shots_pack")
        return d

    def model(self, v, out=None, overwrite=False):
        """The real model V(x, z) ([N, nz], [N, N, nz] in 3D, [N, N_y, nz] on
        parallel lines) from the spectrum v[n_km, nz]; v is used as scratch
        when overwrite is set, else copied."""
        self.upload()
        w = v if overwrite else v.clone()
        if self.n_line:
            shape = (self.n_mid, self.n_line, self.nz)
        elif self.dim == 3:
            shape = (self.n_mid, self.n_mid, self.nz)
        else:
            shape = (self.n_mid, self.nz)
        m = out if out is not None else torch.empty(shape, dtype=torch.float64, device=self.device)
        _lib.check(_lib.load().edt_model(self._h, _ptr(w), _ptr(m), _stream()), "edt_model")
        return m

    def aperture_work(self):
        """A device workspace for aperture_gram (the rows of one frequency)."""
        nb = C.c_size_t(0)
        _lib.check(_lib.load().edt_aperture_work_bytes(self._h, C.byref(nb)), "edt_aperture_work_bytes")
        return torch.empty(max(int(nb.value), 256), dtype=torch.uint8, device=self.device)

    def aperture_gram(self, g64, b_max, out=None, work=None):
        """Finite-aperture Grams (lower triangles) and traces of every pair for
        records kept at |x_R - x_S| <= 2 b_max: (gram[P, nz, nz], trace[P])."""
        self.upload()
        L = _lib.load()
        if work is None:
            work = self.aperture_work()
        if out is None:
            gram = torch.empty(self.n_pairs, self.nz, self.nz, dtype=torch.float64, device=self.device)
            trace = torch.empty(self.n_pairs, dtype=torch.float64, device=self.device)
        else:
            gram, trace = out
        _lib.check(L.edt_aperture_gram(self._h, _ptr(g64), float(b_max), _ptr(gram), _ptr(trace), _ptr(work),
                                       _stream()), "edt_aperture_gram")
        return gram, trace

    def forward(self, g64, v, out=None):
        """Born data rows d_rows[R, 2] (the plan's data type) of the model spectrum v[n_km, nz]."""
        self.upload()
        d = self._rows(out) if out is not None else self._data_rows()
        v = v.to(device=self.device, dtype=torch.complex128).contiguous()
        _lib.check(_lib.load().edt_forward(self._h, _ptr(g64), _ptr(v), _ptr(d), _stream()), "edt_forward")
        return d

    def adjoint(self, vel, g64, d_rows, chol, trace, x, lambda_rel, grad_v, want_d=True,
                want_lambda=True, want_vel=True):
        """(grad_d[R, 2], grad_lambda[1], grad_vel[n_layers]) of a loss with gradient grad_v."""
        self.upload()
        vel = vel.to(device=self.device, dtype=torch.float64).contiguous()
        grad_v = grad_v.to(device=self.device, dtype=torch.complex128).contiguous()
        self._rows(d_rows)
        gd = self._data_rows() if want_d else None
        gl = torch.zeros(1, dtype=torch.float64, device=self.device) if want_lambda else None
        gvel = torch.zeros(self.n_layers, dtype=torch.float64, device=self.device) if want_vel else None
        _lib.check(_lib.load().edt_adjoint(self._h, _ptr(vel), _ptr(g64), _ptr(d_rows), _ptr(chol),
                                           _ptr(trace), _ptr(x), float(lambda_rel), _ptr(grad_v),
                                           _ptr(gd), _ptr(gl), _ptr(gvel), _ptr(self._work), _stream()),
                   "edt_adjoint")
        return gd, gl, gvel

    # -------------------------------------------------------------- timing --
    def timing(self, enable: bool = True):
        _lib.check(_lib.load().edt_timing_enable(self._h, 1 if enable else 0), "edt_timing_enable")

    def timing_read(self):
        """{kernel name: (total ms, launches)} since the previous read."""
        L = _lib.load()
        n = C.c_int(0)
        cap = 64
        names = C.create_string_buffer(32 * cap)
        ms = (C.c_double * cap)()
        cnt = (C.c_int64 * cap)()
        _lib.check(L.edt_timing_read(self._h, cap, names, ms, cnt, C.byref(n)), "edt_timing_read")
        out = {}
        for k in range(min(n.value, cap)):
            nm = names.raw[32 * k:32 * k + 32].split(b"\0", 1)[0].decode()
            out[nm] = (ms[k], int(cnt[k]))
        return out

    # ------------------------------------------------------------ pipeline --
    def run(self, vel, d_rows, lambda_rel, prec="fp64", refine=None, refine_tol=1e-8, max_refine=8):
        """green -> assemble -> solve.  Mixed precisions refine by default."""
        if refine is None:
            refine = prec != "fp64"
        g64, g32 = self.green(vel, want32=prec != "fp64")
        gram, rhs, trace = self.assemble(g64, g32, d_rows, prec)
        x, v, info, steps = self.solve(g64, d_rows, gram, rhs, trace, lambda_rel, refine=refine,
                                       refine_tol=refine_tol, max_refine=max_refine)
        return dict(v=v, x=x, info=info, steps=steps, gram=gram, rhs=rhs, trace=trace, g64=g64, g32=g32)


def solve(survey, d_rows, lambda_rel=None, prec="fp64", **kw):
    """One-shot solve of a survey's data rows; returns V~ (n_km, nz) complex128."""
    p = Plan(survey)
    vel = torch.as_tensor(np.asarray(survey.vel, np.float64), device=p.device)
    lam = survey.lambda_rel if lambda_rel is None else lambda_rel
    return p.run(vel, d_rows, lam, prec=prec, **kw)["v"]
