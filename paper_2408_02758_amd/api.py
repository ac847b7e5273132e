"""Python face of the FTLE library: argument marshalling over the C ABI only.

Every computation runs in the HIP kernels of libftle.so; torch provides device
memory and the current stream.  There is no CPU path.
"""
from __future__ import annotations

import ctypes
from typing import Sequence

import numpy as np
import torch

from . import _lib
from ._lib import FTLEError, check

_DT = {"f32": (_lib.F32, np.float32, torch.float32), "f64": (_lib.F64, np.float64, torch.float64)}


def _stream_handle(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class Mesh:
    """A 2D triangle or 3D tetrahedral mesh prepared for FTLE on the GPU.

    coords: (N, dim) array; cells: (ncells, dim+1) int32 point indices.
    dtype: "f32" or "f64" (storage and arithmetic of every call).
    stencil: "ring1" (all vertices sharing a cell) or "axis" (the 4/6-slot list).
    Mesh.from_csr builds one from a caller-supplied neighbour list instead.
    """

    def __init__(self, coords, cells, dtype: str = "f32", stencil: str = "ring1", reorder: bool = True,
                 tile_log2: int = 0, host_only: bool = False):
        if dtype not in _DT:
            raise ValueError("dtype must be 'f32' or 'f64'")
        L = _lib.load()
        code, npdt, tdt = _DT[dtype]
        coords = np.ascontiguousarray(np.asarray(coords), dtype=npdt)
        cells = np.ascontiguousarray(np.asarray(cells), dtype=np.int32)
        if coords.ndim != 2 or coords.shape[1] not in (2, 3):
            raise ValueError("coords must have shape (N, 2) or (N, 3)")
        dim = coords.shape[1]
        if cells.size and (cells.ndim != 2 or cells.shape[1] != dim + 1):
            raise ValueError(f"cells must have shape (ncells, {dim + 1})")
        flags = {"ring1": _lib.STENCIL_RING1, "axis": _lib.STENCIL_AXIS}[stencil]
        if not reorder:
            flags |= _lib.NO_REORDER
        if host_only:
            flags |= _lib.HOST_ONLY
        flags |= _lib.tile_flag(tile_log2)
        h = ctypes.c_void_p()
        ncells = cells.shape[0] if cells.size else 0
        check(L.ftle_create_mesh(dim, coords.shape[0], coords.ctypes.data, code, ncells,
                                 cells.ctypes.data if ncells else None, flags, ctypes.byref(h)))
        self._init(h, dim, coords.shape[0], dtype, host_only)

    def _init(self, h, dim, n, dtype, host_only):
        code, _, tdt = _DT[dtype]
        self._h = h
        self.dim = dim
        self.n = n
        self.dtype = dtype
        self.torch_dtype = tdt
        self._code = code
        self.host_only = host_only

    @classmethod
    def from_csr(cls, coords, row_ptr, col, dtype: str = "f32", reorder: bool = True, tile_log2: int = 0,
                 host_only: bool = False):
        """Mesh from a caller-supplied stencil: row i of (row_ptr, col) lists the
        neighbours of point i (caller indices, any order; -1 entries and i itself
        are dropped, repeats count twice)."""
        if dtype not in _DT:
            raise ValueError("dtype must be 'f32' or 'f64'")
        L = _lib.load()
        code, npdt, _ = _DT[dtype]
        coords = np.ascontiguousarray(np.asarray(coords), dtype=npdt)
        if coords.ndim != 2 or coords.shape[1] not in (2, 3):
            raise ValueError("coords must have shape (N, 2) or (N, 3)")
        row_ptr = np.ascontiguousarray(np.asarray(row_ptr), dtype=np.int64)
        col = np.ascontiguousarray(np.asarray(col), dtype=np.int32)
        if row_ptr.shape != (coords.shape[0] + 1,):
            raise ValueError("row_ptr must have N+1 entries")
        flags = 0
        if not reorder:
            flags |= _lib.NO_REORDER
        if host_only:
            flags |= _lib.HOST_ONLY
        flags |= _lib.tile_flag(tile_log2)
        h = ctypes.c_void_p()
        check(L.ftle_create_mesh_from_csr(coords.shape[1], coords.shape[0], coords.ctypes.data, code,
                                          row_ptr.ctypes.data, col.ctypes.data if col.size else None, flags,
                                          ctypes.byref(h)))
        m = cls.__new__(cls)
        m._init(h, coords.shape[1], coords.shape[0], dtype, host_only)
        return m

    @classmethod
    def on_device(cls, coords: torch.Tensor, cells: torch.Tensor, stencil: str = "ring1", reorder: bool = True,
                  tile_log2: int = 0, stream=None):
        """Mesh built on the GPU from device tensors (ftle_create_mesh_device):
        coords (N, dim) float32/float64 (the mesh dtype follows it), cells
        (ncells, dim+1) int32, both contiguous on the current device.  The
        stencil ("ring1" or "axis"), the Morton order and the tile records all
        come from kernels; the mesh equals Mesh(coords, cells, stencil=...)
        built on the host."""
        if not (isinstance(coords, torch.Tensor) and coords.is_cuda and coords.is_contiguous()
                and coords.dtype in (torch.float32, torch.float64) and coords.dim() == 2
                and coords.shape[1] in (2, 3)):
            raise ValueError("coords must be a contiguous float32/float64 device tensor of shape (N, 2) or (N, 3)")
        dim = coords.shape[1]
        if not (isinstance(cells, torch.Tensor) and cells.is_cuda and cells.dtype == torch.int32
                and cells.is_contiguous() and cells.dim() == 2 and cells.shape[1] == dim + 1):
            raise ValueError(f"cells must be a contiguous int32 device tensor of shape (ncells, {dim + 1})")
        dtype = "f64" if coords.dtype == torch.float64 else "f32"
        flags = _lib.tile_flag(tile_log2) | {"ring1": _lib.STENCIL_RING1, "axis": _lib.STENCIL_AXIS}[stencil]
        if not reorder:
            flags |= _lib.NO_REORDER
        h = ctypes.c_void_p()
        ncells = cells.shape[0]
        check(_lib.load().ftle_create_mesh_device(dim, coords.shape[0], ctypes.c_void_p(coords.data_ptr()),
                                                  _DT[dtype][0], ncells,
                                                  ctypes.c_void_p(cells.data_ptr()) if ncells else None, flags,
                                                  _stream_handle(stream), ctypes.byref(h)))
        m = cls.__new__(cls)
        m._init(h, dim, coords.shape[0], dtype, False)
        return m

    @classmethod
    def from_csr_on_device(cls, coords: torch.Tensor, row_ptr: torch.Tensor, col: torch.Tensor, reorder: bool = True,
                           tile_log2: int = 0, stream=None):
        """Mesh.from_csr built on the GPU (ftle_create_mesh_device_from_csr):
        coords (N, dim) float32/float64, row_ptr (N+1,) int64 and col int32
        device tensors (caller indices; -1 and self entries dropped, repeats
        kept), e.g. ring1_csr's output or the paper's list with
        row_ptr = 2*dim*arange(N+1)."""
        if not (isinstance(coords, torch.Tensor) and coords.is_cuda and coords.is_contiguous()
                and coords.dtype in (torch.float32, torch.float64) and coords.dim() == 2
                and coords.shape[1] in (2, 3)):
            raise ValueError("coords must be a contiguous float32/float64 device tensor of shape (N, 2) or (N, 3)")
        n, dim = coords.shape
        if not (row_ptr.is_cuda and row_ptr.dtype == torch.int64 and row_ptr.is_contiguous()
                and tuple(row_ptr.shape) == (n + 1,)):
            raise ValueError("row_ptr must be a contiguous int64 device tensor of N+1 entries")
        if not (col.is_cuda and col.dtype == torch.int32 and col.is_contiguous()):
            raise ValueError("col must be a contiguous int32 device tensor")
        dtype = "f64" if coords.dtype == torch.float64 else "f32"
        flags = _lib.tile_flag(tile_log2)
        if not reorder:
            flags |= _lib.NO_REORDER
        h = ctypes.c_void_p()
        check(_lib.load().ftle_create_mesh_device_from_csr(
            dim, n, ctypes.c_void_p(coords.data_ptr()), _DT[dtype][0], ctypes.c_void_p(row_ptr.data_ptr()),
            ctypes.c_void_p(col.data_ptr()) if col.numel() else None, flags, _stream_handle(stream),
            ctypes.byref(h)))
        m = cls.__new__(cls)
        m._init(h, dim, n, dtype, False)
        return m

    # -- lifetime ---------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().ftle_destroy_mesh(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass

    @property
    def handle(self):
        return self._h

    # -- host-side accessors ------------------------------------------------
    def info(self):
        d, n, nnz, dt = ctypes.c_int(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int()
        check(_lib.load().ftle_mesh_info(self._h, ctypes.byref(d), ctypes.byref(n), ctypes.byref(nnz),
                                         ctypes.byref(dt)))
        return {"dim": d.value, "n": n.value, "nnz": nnz.value, "dtype": "f64" if dt.value else "f32"}

    def csr(self):
        """(row_ptr, col, perm) in Morton order (col holds Morton positions)."""
        nnz = self.info()["nnz"]
        row_ptr = np.empty(self.n + 1, np.int32)
        col = np.empty(max(nnz, 1), np.int32)
        perm = np.empty(self.n, np.int32)
        check(_lib.load().ftle_mesh_get_csr(self._h, row_ptr.ctypes.data, col.ctypes.data, perm.ctypes.data))
        return row_ptr, col[:nnz], perm

    def tile_stats(self):
        vals = [ctypes.c_int64() for _ in range(4)]
        check(_lib.load().ftle_mesh_tile_stats(self._h, *[ctypes.byref(v) for v in vals]))
        return dict(zip(["n_tiles", "max_tile_points", "halo_entries", "record_bytes"], [v.value for v in vals]))

    def tile_records(self, adjoint: bool = False):
        """Raw tile records, one dict per tile: P, H and the record's arrays
        (words, runs, smask, xmask, spre, xpre, xlast, xend)."""
        L = _lib.load()
        nt, rb = ctypes.c_int64(), ctypes.c_int64()
        check(L.ftle_mesh_get_tiles(self._h, int(adjoint), ctypes.byref(nt), ctypes.byref(rb), None, None))
        meta = np.empty((nt.value, 4), np.uint32)
        rec = np.empty(max(rb.value // 4, 1), np.uint32)
        check(L.ftle_mesh_get_tiles(self._h, int(adjoint), None, None, meta.ctypes.data, rec.ctypes.data))
        h16 = meta.view(np.uint16).reshape(-1, 8)
        out = []
        for t in range(nt.value):
            P, H, nw, nr, nx = (int(v) for v in h16[t, 2:7])
            G, Q = (P + H + 31) // 32, (P + 31) // 32
            b = int(meta[t, 0]) * 16   # byte offset
            o_runs = 4 * nw
            o_smask = o_runs + 4 * nr
            o_xmask = o_smask + 4 * G
            o_spre = o_xmask + 4 * Q
            o_xpre = o_spre + 2 * G
            o_xlast = o_xpre + 2 * Q
            o_xend = o_xlast + 2 * Q
            by = rec.view(np.uint8)

            def arr(off, cnt, dt):
                size = np.dtype(dt).itemsize
                return by[b + off:b + off + cnt * size].view(dt).copy()

            out.append(dict(P=P, H=H, nwf=int(h16[t, 7]), words=arr(0, nw, np.uint32),
                            runs=arr(o_runs, nr, np.uint32), smask=arr(o_smask, G, np.uint32),
                            xmask=arr(o_xmask, Q, np.uint32), spre=arr(o_spre, G, np.uint16),
                            xpre=arr(o_xpre, Q, np.uint16), xlast=arr(o_xlast, Q, np.uint16),
                            xend=arr(o_xend, nx, np.uint16)))
        return out

    def tiles(self, adjoint: bool = False):
        """Tile records decoded: list of (idx uint32[P+H], rowend uint16[P],
        entries uint16[3 nwf], P, H).

        idx is the caller index of every staged slot; entries are the
        neighbours' local indices (slots), three per stencil word, each row
        padded to a multiple of 3 with the point's own slot; rowend counts
        words.  Rows that the record stores as shifts of an earlier row are
        expanded."""
        out = []
        for r in self.tile_records(adjoint):
            P, H = r["P"], r["H"]
            S = P + H
            bits = lambda m, k: ((m[:, None] >> np.arange(32, dtype=np.uint32)) & 1).reshape(-1)[:k].astype(bool)
            starts = bits(r["smask"], S)
            run_of = np.cumsum(starts) - 1
            idx = (r["runs"][run_of].astype(np.uint64) + np.arange(S, dtype=np.uint64)) % (1 << 32)
            w = r["words"]
            ent_x = np.stack([w & 0x3FF, (w >> 10) & 0x3FF, (w >> 20) & 0x3FF], 1).reshape(-1).astype(np.int64)
            xend = r["xend"].astype(np.int64)
            expl = np.flatnonzero(bits(r["xmask"], P))
            rows, ends, pos = [], [], 0
            k = -1
            for l in range(P):
                if k + 1 < len(expl) and expl[k + 1] == l:
                    k += 1
                a = int(expl[k])
                s0 = int(xend[k - 1]) if k else 0
                rows.append(ent_x[3 * s0:3 * int(xend[k])] + (l - a))
                pos += len(rows[-1]) // 3
                ends.append(pos)
            ent = np.concatenate(rows).astype(np.uint16) if rows else np.zeros(0, np.uint16)
            out.append((idx.astype(np.uint32), np.array(ends, np.uint16), ent, P, H))
        return out

    def set_blocks(self, fwd: int = 0, adjoint: int = 0):
        check(_lib.load().ftle_mesh_set_blocks(self._h, int(fwd), int(adjoint)))

    def blocks(self):
        """(forward, adjoint) threads per workgroup."""
        f, a = ctypes.c_int(), ctypes.c_int()
        check(_lib.load().ftle_mesh_get_blocks(self._h, ctypes.byref(f), ctypes.byref(a)))
        return f.value, a.value

    def tape_bytes(self) -> int:
        b = ctypes.c_int64()
        check(_lib.load().ftle_tape_bytes(self._h, ctypes.byref(b)))
        return b.value

    # -- device calls -------------------------------------------------------
    def _check_flow(self, t: torch.Tensor, name="flow", shape=None):
        shape = (self.n, self.dim) if shape is None else shape
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a CUDA (HIP) tensor")
        if t.dtype != self.torch_dtype:
            raise TypeError(f"{name} must have dtype {self.torch_dtype}")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} must have shape {shape}, got {tuple(t.shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")

    def forward(self, flow: torch.Tensor, T: float, out: torch.Tensor | None = None, stream=None):
        self._check_flow(flow)
        if out is None:
            out = torch.empty(self.n, dtype=self.torch_dtype, device=flow.device)
        self._check_flow(out, "out", (self.n,))
        check(_lib.load().ftle_forward(self._h, ctypes.c_void_p(flow.data_ptr()), self._code, float(T),
                                       ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
        return out

    def encode_flow_f16(self, flow: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """binary16(phi - x), the half-precision storage of a float32 flow map
        (2D float32 meshes; ftle_encode_flow_f16)."""
        self._check_flow(flow)
        if out is None:
            out = torch.empty(self.n, 2, dtype=torch.float16, device=flow.device)
        if not (out.is_cuda and out.dtype == torch.float16 and out.is_contiguous() and tuple(out.shape) == (self.n, 2)):
            raise ValueError(f"out must be a contiguous float16 device tensor of shape ({self.n}, 2)")
        check(_lib.load().ftle_encode_flow_f16(self._h, ctypes.c_void_p(flow.data_ptr()),
                                               ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
        return out

    def forward_f16(self, delta: torch.Tensor, T: float, out: torch.Tensor | None = None, stream=None):
        """Float32 FTLE of the flow map x + delta, delta the binary16
        displacements encode_flow_f16 writes (ftle_forward_f16)."""
        if not (isinstance(delta, torch.Tensor) and delta.is_cuda and delta.dtype == torch.float16
                and delta.is_contiguous() and tuple(delta.shape) == (self.n, 2)):
            raise ValueError(f"delta must be a contiguous float16 device tensor of shape ({self.n}, 2)")
        if out is None:
            out = torch.empty(self.n, dtype=torch.float32, device=delta.device)
        self._check_flow(out, "out", (self.n,))
        check(_lib.load().ftle_forward_f16(self._h, ctypes.c_void_p(delta.data_ptr()), float(T),
                                           ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
        return out

    def forward_tape(self, flow: torch.Tensor, T: float, out=None, tape=None, stream=None):
        self._check_flow(flow)
        if out is None:
            out = torch.empty(self.n, dtype=self.torch_dtype, device=flow.device)
        if tape is None:
            tape = torch.empty(self.n * (2 * self.dim + 1), dtype=self.torch_dtype, device=flow.device)
        self._check_flow(out, "out", (self.n,))
        self._check_flow(tape, "tape", (self.n * (2 * self.dim + 1),))
        check(_lib.load().ftle_forward_tape(self._h, ctypes.c_void_p(flow.data_ptr()), self._code, float(T),
                                            ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(tape.data_ptr()),
                                            _stream_handle(stream)))
        return out, tape

    def backward_tape(self, tape: torch.Tensor, grad_ftle: torch.Tensor, grad_flow=None, stream=None):
        self._check_flow(tape, "tape", (self.n * (2 * self.dim + 1),))
        self._check_flow(grad_ftle, "grad_ftle", (self.n,))
        if grad_flow is None:
            grad_flow = torch.empty(self.n, self.dim, dtype=self.torch_dtype, device=tape.device)
        self._check_flow(grad_flow, "grad_flow")
        check(_lib.load().ftle_backward_tape(self._h, ctypes.c_void_p(tape.data_ptr()), self._code,
                                             ctypes.c_void_p(grad_ftle.data_ptr()),
                                             ctypes.c_void_p(grad_flow.data_ptr()), _stream_handle(stream)))
        return grad_flow

    def backward(self, flow: torch.Tensor, T: float, grad_ftle: torch.Tensor, grad_flow=None, stream=None):
        self._check_flow(flow)
        self._check_flow(grad_ftle, "grad_ftle", (self.n,))
        if grad_flow is None:
            grad_flow = torch.empty(self.n, self.dim, dtype=self.torch_dtype, device=flow.device)
        self._check_flow(grad_flow, "grad_flow")
        check(_lib.load().ftle_backward(self._h, ctypes.c_void_p(flow.data_ptr()), self._code, float(T),
                                        ctypes.c_void_p(grad_ftle.data_ptr()),
                                        ctypes.c_void_p(grad_flow.data_ptr()), _stream_handle(stream)))
        return grad_flow

    def backward_noalloc(self, flow: torch.Tensor, T: float, grad_ftle: torch.Tensor, grad_flow: torch.Tensor,
                         stream=None):
        """ftle_backward with its tape in the library's fixed per-GPU scratch:
        the call allocates nothing (grad_flow must be given).  Calls that
        overlap on one GPU race; order them on one stream."""
        self._check_flow(flow)
        self._check_flow(grad_ftle, "grad_ftle", (self.n,))
        self._check_flow(grad_flow, "grad_flow")
        check(_lib.load().ftle_backward_noalloc(self._h, ctypes.c_void_p(flow.data_ptr()), self._code, float(T),
                                                ctypes.c_void_p(grad_ftle.data_ptr()),
                                                ctypes.c_void_p(grad_flow.data_ptr()), _stream_handle(stream)))
        return grad_flow

    def fp64_hits(self, reset: bool = False) -> int:
        h = ctypes.c_int64()
        check(_lib.load().ftle_mesh_fp64_hits(self._h, ctypes.byref(h), int(reset)))
        return h.value


def _handles(meshes: Sequence[Mesh]):
    arr = (ctypes.c_void_p * len(meshes))(*[m.handle.value for m in meshes])
    return arr


def batched(meshes: Sequence[Mesh], flows: Sequence[torch.Tensor], Ts: Sequence[float], outs=None, stream=None):
    """One launch over many meshes (a persistent grid draining a queue or a
    flat grid, as autotuned or pinned), replayed from a cached HIP graph."""
    n = len(meshes)
    if not (len(flows) == n == len(Ts)):
        raise ValueError("meshes, flows and Ts must have the same length")
    if n == 0:
        return []
    for m, f in zip(meshes, flows):
        m._check_flow(f)
    if outs is None:
        outs = [torch.empty(m.n, dtype=m.torch_dtype, device=f.device) for m, f in zip(meshes, flows)]
    for m, o in zip(meshes, outs):
        m._check_flow(o, "out", (m.n,))
    fl = (ctypes.c_void_p * n)(*[f.data_ptr() for f in flows])
    ou = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
    ts = (ctypes.c_double * n)(*[float(t) for t in Ts])
    check(_lib.load().ftle_batched(n, _handles(meshes), fl, ts, ou, meshes[0]._code, _stream_handle(stream)))
    return outs


class BatchedCall:
    """A batched forward call prepared once: validates and marshals the meshes,
    flow maps, times and outputs a single time, then launches with one C call
    per __call__ (for serving loops and benchmarks that reuse their buffers).
    Holds references to the tensors it was built with."""

    def __init__(self, meshes: Sequence[Mesh], flows: Sequence[torch.Tensor], Ts: Sequence[float], outs=None):
        n = len(meshes)
        if not (len(flows) == n == len(Ts)) or n == 0:
            raise ValueError("meshes, flows and Ts must be non-empty and of the same length")
        for m, f in zip(meshes, flows):
            m._check_flow(f)
        if outs is None:
            outs = [torch.empty(m.n, dtype=m.torch_dtype, device=f.device) for m, f in zip(meshes, flows)]
        for m, o in zip(meshes, outs):
            m._check_flow(o, "out", (m.n,))
        self.meshes, self.flows, self.outs = list(meshes), list(flows), list(outs)
        self._n = n
        self._h = _handles(meshes)
        self._fl = (ctypes.c_void_p * n)(*[f.data_ptr() for f in flows])
        self._ou = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
        self._ts = (ctypes.c_double * n)(*[float(t) for t in Ts])
        self._code = meshes[0]._code
        self._fn = _lib.load().ftle_batched

    def __call__(self, stream=None):
        check(self._fn(self._n, self._h, self._fl, self._ts, self._ou, self._code, _stream_handle(stream)))
        return self.outs


def batched_config(meshes: Sequence[Mesh]):
    b, k, g = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    check(_lib.load().ftle_batched_config(len(meshes), _handles(meshes), ctypes.byref(b), ctypes.byref(k),
                                          ctypes.byref(g)))
    return {"block": b.value, "tiles_per_pop": k.value, "grid": g.value}


class FTLEFunction(torch.autograd.Function):
    """FTLE with a hand-written adjoint: forward records a tape, backward gathers dL/dflow."""

    @staticmethod
    def forward(ctx, flow, mesh: Mesh, T: float):
        out, tape = mesh.forward_tape(flow.contiguous(), T)
        ctx.mesh = mesh
        ctx.tape = tape
        return out

    @staticmethod
    def backward(ctx, grad_out):
        grad = ctx.mesh.backward_tape(ctx.tape, grad_out.contiguous())
        ctx.tape = None
        return grad, None, None


_FLOWS = {"double_gyre": (0, 2), "abc": (1, 3)}


def _check_out(out, shape, dtype, name="out", not_alias=None):
    """out must be a contiguous device tensor of the given shape and dtype (and
    not the input not_alias): the kernels write exactly that many values."""
    if not (isinstance(out, torch.Tensor) and out.is_cuda and out.dtype == dtype and out.is_contiguous()
            and tuple(out.shape) == tuple(shape)):
        raise ValueError(f"{name} must be a contiguous {dtype} device tensor of shape {tuple(shape)}")
    if not_alias is not None and out.numel() and out.data_ptr() == not_alias.data_ptr():
        raise ValueError(f"{name} must not be the input tensor")


def advect_rk4(flow: str, x0: torch.Tensor, t0, T, dt: float, params=None, out: torch.Tensor | None = None,
               stream=None) -> torch.Tensor:
    """Flow map x(t0 + T) of particles at x0 (device tensor, (N, 2) for
    "double_gyre" or (N, 3) for "abc", float32 or float64) by RK4 on the GPU.
    t0 and T: floats, or float64 device tensors of N per-particle values."""
    kind, dim = _FLOWS[flow]
    if not (x0.is_cuda and x0.is_contiguous() and x0.dim() == 2 and x0.shape[1] == dim):
        raise ValueError(f"x0 must be a contiguous device tensor of shape (N, {dim})")
    code = {torch.float32: 0, torch.float64: 1}.get(x0.dtype)
    if code is None:
        raise ValueError("x0 must be float32 or float64")
    n = x0.shape[0]

    def per_point(v, name):
        if isinstance(v, torch.Tensor):
            if not (v.is_cuda and v.dtype == torch.float64 and v.is_contiguous() and v.shape == (n,)):
                raise ValueError(f"{name} must be a contiguous float64 device tensor of {n} values")
            return ctypes.c_void_p(v.data_ptr()), 0.0
        return None, float(v)

    t0p, t0s = per_point(t0, "t0")
    Tp, Ts = per_point(T, "T")
    if out is None:
        out = torch.empty_like(x0)
    _check_out(out, x0.shape, x0.dtype, not_alias=x0)
    prm = None if params is None else (ctypes.c_double * 3)(*[float(v) for v in params])
    check(_lib.load().ftle_advect_rk4(kind, prm, n, ctypes.c_void_p(x0.data_ptr()), code, t0p, Tp, t0s, Ts,
                                      float(dt), ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
    return out


def advect_rk4_grid(velocity: torch.Tensor, origin, spacing, t_first: float, t_step: float, x0: torch.Tensor, t0, T,
                    dt: float, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Flow map x(t0 + T) of particles at x0 by RK4 on the GPU in a velocity
    field sampled on a regular grid (ftle_advect_rk4_grid): velocity is a
    contiguous float32/float64 device tensor (n_times, [nz,] ny, nx, dim) of
    the velocity at node origin + index * spacing (x fastest) and time
    t_first + k * t_step; multilinear in space, linear in time, the nearest box
    point and slice outside.  x0 (N, dim), t0 and T as in advect_rk4."""
    if not (isinstance(velocity, torch.Tensor) and velocity.is_cuda and velocity.is_contiguous()
            and velocity.dtype in (torch.float32, torch.float64) and velocity.dim() in (4, 5)):
        raise ValueError("velocity must be a contiguous float32/float64 device tensor (n_times, [nz,] ny, nx, dim)")
    dim = velocity.shape[-1]
    if velocity.dim() != dim + 2:
        raise ValueError("velocity's last axis must hold dim components for a dim-dimensional grid")
    if not (x0.is_cuda and x0.is_contiguous() and x0.dim() == 2 and x0.shape[1] == dim
            and x0.dtype in (torch.float32, torch.float64)):
        raise ValueError(f"x0 must be a contiguous float32/float64 device tensor of shape (N, {dim})")
    n = x0.shape[0]

    def per_point(v, name):
        if isinstance(v, torch.Tensor):
            if not (v.is_cuda and v.dtype == torch.float64 and v.is_contiguous() and v.shape == (n,)):
                raise ValueError(f"{name} must be a contiguous float64 device tensor of {n} values")
            return ctypes.c_void_p(v.data_ptr()), 0.0
        return None, float(v)

    t0p, t0s = per_point(t0, "t0")
    Tp, Ts = per_point(T, "T")
    if out is None:
        out = torch.empty_like(x0)
    _check_out(out, x0.shape, x0.dtype, not_alias=x0)
    if len(origin) != dim or len(spacing) != dim:
        raise ValueError(f"origin and spacing need {dim} values each")
    shape = (ctypes.c_int64 * dim)(*[int(v) for v in velocity.shape[1:-1][::-1]])
    org = (ctypes.c_double * dim)(*[float(v) for v in origin])
    spc = (ctypes.c_double * dim)(*[float(v) for v in spacing])
    check(_lib.load().ftle_advect_rk4_grid(
        dim, shape, org, spc, velocity.shape[0], float(t_first), float(t_step), ctypes.c_void_p(velocity.data_ptr()),
        1 if velocity.dtype == torch.float64 else 0, n, ctypes.c_void_p(x0.data_ptr()),
        1 if x0.dtype == torch.float64 else 0, t0p, Tp, t0s, Ts, float(dt), ctypes.c_void_p(out.data_ptr()),
        _stream_handle(stream)))
    return out


def ring1_workspace_bytes(dim: int, n_points: int, n_cells: int) -> int:
    """Device workspace bytes of ring1_csr(..., workspace=...) (ftle_ring1_csr_workspace)."""
    b = ctypes.c_int64()
    check(_lib.load().ftle_ring1_csr_workspace(dim, int(n_points), int(n_cells), ctypes.byref(b)))
    return b.value


def ring1_csr(dim: int, n_points: int, cells: torch.Tensor, stream=None, workspace: torch.Tensor | None = None,
              col: torch.Tensor | None = None):
    """The one-ring stencil of a cell mesh built on the GPU (ftle_ring1_csr):
    cells is a contiguous int32 device tensor (n_cells, dim + 1); returns
    (row_ptr int64 (n_points + 1,), col int32 (nnz,)) on the same device,
    every other point sharing a cell with point i, ascending, once each.
    workspace: a device tensor of at least ring1_workspace_bytes bytes to use
    instead of an allocation inside the call (ftle_ring1_csr_ws); col: the
    output buffer (int32, its size the capacity).  Mesh.from_csr takes the
    result (on the host) to build the mesh."""
    if not (cells.is_cuda and cells.dtype == torch.int32 and cells.is_contiguous() and cells.dim() == 2
            and cells.shape[1] == dim + 1):
        raise ValueError(f"cells must be a contiguous int32 device tensor of shape (n_cells, {dim + 1})")
    n_cells = cells.shape[0]
    row_ptr = torch.empty(int(n_points) + 1, dtype=torch.int64, device=cells.device)
    if col is None:
        col = torch.empty(max(1, n_cells * dim * (dim + 1)), dtype=torch.int32, device=cells.device)
    if not (col.is_cuda and col.dtype == torch.int32 and col.is_contiguous()):
        raise ValueError("col must be a contiguous int32 device tensor")
    nnz = ctypes.c_int64(0)
    L = _lib.load()
    args = [dim, int(n_points), n_cells, ctypes.c_void_p(cells.data_ptr()), ctypes.c_void_p(row_ptr.data_ptr()),
            ctypes.c_void_p(col.data_ptr()), col.numel(), ctypes.byref(nnz)]
    if workspace is None:
        check(L.ftle_ring1_csr(*args, _stream_handle(stream)))
    else:
        if not (workspace.is_cuda and workspace.is_contiguous()):
            raise ValueError("workspace must be a contiguous device tensor")
        check(L.ftle_ring1_csr_ws(*args, ctypes.c_void_p(workspace.data_ptr()),
                                  workspace.numel() * workspace.element_size(), _stream_handle(stream)))
    return row_ptr, col[:nnz.value]


def _device_points(t: torch.Tensor, name: str, n: int, dim: int):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous() and t.dtype in (torch.float32, torch.float64)
            and tuple(t.shape) == (n, dim)):
        raise ValueError(f"{name} must be a contiguous float32/float64 device tensor of shape ({n}, {dim})")


def axis_ell(coords: torch.Tensor, row_ptr: torch.Tensor, col: torch.Tensor, stream=None) -> torch.Tensor:
    """The paper's fixed-width list (n, 2*dim) int32 built on the GPU from a
    one-ring stencil (ftle_axis_ell): per signed axis direction the neighbour
    with the largest cosine, -1 where there is none."""
    n, dim = coords.shape
    _device_points(coords, "coords", n, dim)
    if not (row_ptr.is_cuda and row_ptr.dtype == torch.int64 and row_ptr.is_contiguous() and row_ptr.shape == (n + 1,)):
        raise ValueError("row_ptr must be a contiguous int64 device tensor of n+1 entries")
    if not (col.is_cuda and col.dtype == torch.int32 and col.is_contiguous()):
        raise ValueError("col must be a contiguous int32 device tensor")
    ell = torch.empty(n, 2 * dim, dtype=torch.int32, device=coords.device)
    code = _lib.F64 if coords.dtype == torch.float64 else _lib.F32
    check(_lib.load().ftle_axis_ell(dim, n, ctypes.c_void_p(coords.data_ptr()), code,
                                    ctypes.c_void_p(row_ptr.data_ptr()), ctypes.c_void_p(col.data_ptr()),
                                    ctypes.c_void_p(ell.data_ptr()), _stream_handle(stream)))
    return ell


def forward_ell(coords: torch.Tensor, ell: torch.Tensor, flow: torch.Tensor, T: float, staged: bool = False,
                out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """FTLE from the paper's fixed-width list (ftle_forward_ell): coords and
    flow (n, dim) device tensors of one dtype, ell (n, 2*dim) int32 (-1 where
    absent).  staged: each workgroup's block of points staged in LDS."""
    n, dim = coords.shape
    _device_points(coords, "coords", n, dim)
    _device_points(flow, "flow", n, dim)
    if flow.dtype != coords.dtype:
        raise ValueError("flow and coords must have the same dtype")
    if not (ell.is_cuda and ell.dtype == torch.int32 and ell.is_contiguous() and tuple(ell.shape) == (n, 2 * dim)):
        raise ValueError(f"ell must be a contiguous int32 device tensor of shape ({n}, {2 * dim})")
    if out is None:
        out = torch.empty(n, dtype=coords.dtype, device=coords.device)
    _check_out(out, (n,), coords.dtype)
    code = _lib.F64 if coords.dtype == torch.float64 else _lib.F32
    check(_lib.load().ftle_forward_ell(dim, n, ctypes.c_void_p(coords.data_ptr()), code,
                                       ctypes.c_void_p(ell.data_ptr()), ctypes.c_void_p(flow.data_ptr()), float(T),
                                       ctypes.c_void_p(out.data_ptr()),
                                       _lib.ELL_STAGED if staged else _lib.ELL_DIRECT, _stream_handle(stream)))
    return out


def cached_memory_bytes() -> int:
    """Device memory the mesh builds keep between calls (all devices)."""
    v = ctypes.c_int64(0)
    check(_lib.load().ftle_cached_memory_bytes(ctypes.byref(v)))
    return v.value


def release_cached_memory() -> None:
    """Free the device memory the mesh builds keep between calls."""
    check(_lib.load().ftle_release_cached_memory())


def force_wide_offsets(on: bool) -> None:
    """Testing aid: make every later launch take the 64-bit offset path (see ftle_force_wide_offsets)."""
    check(_lib.load().ftle_force_wide_offsets(int(bool(on))))


def set_eig_threshold(tau: float) -> None:
    """Testing aid: threshold of the 3D float32 eigenvalue recompute (r + 1 < tau
    goes through float64; tau > 2 sends every point, 0 none, < 0 restores the
    default; see ftle_set_eig_threshold)."""
    check(_lib.load().ftle_set_eig_threshold(float(tau)))


def eig_threshold() -> float:
    t = ctypes.c_double()
    check(_lib.load().ftle_get_eig_threshold(ctypes.byref(t)))
    return t.value


def pin_batched_config(block: int = 0, tiles_per_pop: int = 0, per_cu_cap: int = 0) -> None:
    """Testing aid: pin the batched launch shape (block 0 unpins; tiles_per_pop 0
    is the flat grid; see ftle_batched_pin_config)."""
    check(_lib.load().ftle_batched_pin_config(int(block), int(tiles_per_pop), int(per_cu_cap)))


def ftle(mesh: Mesh, flow: torch.Tensor, T: float) -> torch.Tensor:
    """Differentiable FTLE of a flow map on a mesh."""
    return FTLEFunction.apply(flow, mesh, T)


__all__ = ["Mesh", "batched", "BatchedCall", "batched_config", "FTLEFunction", "ftle", "FTLEError",
           "force_wide_offsets", "set_eig_threshold", "eig_threshold", "pin_batched_config", "advect_rk4",
           "advect_rk4_grid", "ring1_csr", "ring1_workspace_bytes", "axis_ell", "forward_ell",
           "cached_memory_bytes", "release_cached_memory"]
