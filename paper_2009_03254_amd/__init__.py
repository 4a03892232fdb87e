"""bcmc: GPU-driven isosurface extraction from block-compressed volumes on
MI355X (gfx950) -- Usher & Pascucci, arXiv 2009.03254, Sec. 4.

A thin Python binding of the C ABI in ``include/bcmc.h`` (libbcmc.so, built
in-tree by ``paper_2009_03254_amd.build``).  It only marshals arguments: every
step of the extraction runs in the library's HIP kernels.  PyTorch supplies
device memory and the current HIP stream.

    import torch, paper_2009_03254_amd as bcmc
    stream = bcmc.encode(field_cuda, rate=8)          # fixed-rate ZFP on the GPU
    vol = bcmc.Volume(stream, field_cuda.shape[::-1], "f32", 8)
    vol.set_cache_budget(initial_bytes=vol.n_blocks * 64)
    verts, T = vol.extract(0.5)       # [3T, 4] int32 rows: x, y, z (float bits), block
    xyz, blk = bcmc.split_vertices(verts)
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import _capi
from ._capi import BcmcError, lib  # noqa: F401

__all__ = ["Volume", "FieldVolume", "Batch", "ExtractFn", "encode", "mc_table", "num_blocks",
           "blocks_from_field", "split_vertices", "global_positions", "edge8_positions",
           "VERTEX_F32", "VERTEX_EDGE8", "VERTEX_Q10", "q10_positions", "vertices_to_q10",
           "BcmcError", "lib"]

F32, F64 = 0, 1
VERTEX_F32, VERTEX_EDGE8, VERTEX_Q10 = 0, 1, 2     # record formats of Volume.extract
_TYPES = {"f32": F32, "float32": F32, "f64": F64, "float64": F64}


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _dev_ptr(t):
    return C.c_void_p(t.data_ptr())


def num_blocks(nx, ny, nz):
    return int(lib().bcmc_num_blocks(nx, ny, nz))


def mc_table():
    """The library's generated marching cubes table as
    (num_tris[256], tris[256,16] edge ids padded with -1)."""
    packed = np.zeros(256, dtype=np.uint64)
    _capi.check(lib().bcmc_mc_table(packed.ctypes.data_as(C.c_void_p)))
    nt = (packed >> np.uint64(60)).astype(np.int32)
    tri = np.full((256, 16), -1, dtype=np.int32)
    for c in range(256):
        w = int(packed[c])
        for k in range(3 * int(nt[c])):
            tri[c, k] = (w >> (4 * k)) & 15
    return nt, tri


def encode(field, rate, stream=None, out=None):
    """Fixed-rate ZFP compression of a CUDA tensor [nz, ny, nx] (float32 or
    float64) -> CUDA uint64 tensor of N_b*rate words (into `out` when
    given)."""
    torch = _torch()
    if not field.is_cuda:
        raise ValueError("encode expects a CUDA tensor")
    field = field.contiguous()
    if field.dtype == torch.float32:
        typ = F32
    elif field.dtype == torch.float64:
        typ = F64
    else:
        raise TypeError("field must be float32 or float64")
    nz, ny, nx = field.shape
    n_words = num_blocks(nx, ny, nz) * rate
    if out is None:
        out = torch.empty(n_words, dtype=torch.uint64, device=field.device)
    elif out.numel() != n_words or not out.is_cuda or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous CUDA tensor of {n_words} words")
    _capi.check(lib().bcmc_encode(_dev_ptr(field), typ, nx, ny, nz, rate, _dev_ptr(out),
                                  _stream_ptr(stream)))
    return out


def blocks_from_field(field):
    """[nz, ny, nx] CUDA tensor -> [N_b, 64] block layout (block id
    bx + nbx*(by + nby*bz), sample lx + 4*ly + 16*lz), partial blocks padded
    by replicating the last sample (a pure layout change)."""
    torch = _torch()
    nz, ny, nx = field.shape
    pz, py, px = (-nz) % 4, (-ny) % 4, (-nx) % 4
    f = field
    if px or py or pz:
        f = torch.nn.functional.pad(f[None, None], (0, px, 0, py, 0, pz), mode="replicate")[0, 0]
    nbz, nby, nbx = f.shape[0] // 4, f.shape[1] // 4, f.shape[2] // 4
    f = f.reshape(nbz, 4, nby, 4, nbx, 4).permute(0, 2, 4, 1, 3, 5)
    return f.reshape(-1, 64).contiguous()


def split_vertices(verts):
    """[n, 4] int32 records -> (xyz float32 [n, 3] view, block int32 [n] view)."""
    torch = _torch()
    return verts.view(torch.float32)[:, :3], verts[:, 3]


def edge8_positions(records, dims=None, dtype=None):
    """Decode 8-byte edge records ([n] int64 CUDA tensor) into block-relative
    positions [n, 3] (the edge's first corner plus (q + 0.5) / 2^22 along its
    axis; float64 by default) and block ids [n] (int64); with dims, global
    voxel coordinates instead of block-relative ones."""
    torch = _torch()
    r = records.to(torch.int64)
    block = r & 0xFFFFFFFF
    cell = (r >> 32) & 63
    e = (r >> 38) & 15
    q = (r >> 42) & ((1 << 22) - 1)
    axis = e >> 2
    b0, b1 = e & 1, (e >> 1) & 1
    zero = torch.zeros_like(e)
    off = torch.stack([torch.where(axis == 0, zero, b0),
                       torch.where(axis == 1, zero, torch.where(axis == 0, b0, b1)),
                       torch.where(axis == 2, zero, b1)], dim=1)
    corner = torch.stack([cell & 3, (cell >> 2) & 3, cell >> 4], dim=1) + off
    dt = dtype or torch.float64
    pos = corner.to(dt)
    pos[torch.arange(r.numel(), device=r.device), axis] += (q.to(dt) + 0.5) / 4194304.0
    if dims is not None:
        pos = global_positions(pos, block, dims, dtype=dt)
    return pos, block


def q10_positions(records, dims=None, dtype=None):
    """Dequantise the paper's 8-byte vertices ([n] int64 CUDA tensor, 10-bit
    block-relative coordinates in the low 32 bits, block id in the high 32):
    positions q * 4 / 1023 [n, 3] (float32 by default) and block ids [n]
    (int64); with dims, global voxel coordinates."""
    torch = _torch()
    r = records.to(torch.int64)
    code = r & 0xFFFFFFFF
    block = (r >> 32) & 0xFFFFFFFF
    dt = dtype or torch.float32
    q = torch.stack([code & 1023, (code >> 10) & 1023, (code >> 20) & 1023], dim=1)
    pos = q.to(dt) * (4.0 / 1023.0)
    if dims is not None:
        pos = global_positions(pos, block, dims, dtype=dt)
    return pos, block


def vertices_to_q10(verts, out=None, stream=None):
    """16-byte vertex records ([n, 4] int32 CUDA tensor) -> the paper's 8-byte
    records ([n] int64), on the GPU."""
    torch = _torch()
    n = verts.shape[0]
    if out is None:
        out = torch.empty(max(n, 1), dtype=torch.int64, device=verts.device)
    verts = verts.contiguous()
    _capi.check(lib().bcmc_vertices_to_q10(_dev_ptr(verts) if n else None, n,
                                           _dev_ptr(out) if n else None, _stream_ptr(stream)))
    return out[:n]


def global_positions(xyz, block, dims, dtype=None):
    """Block-relative positions + block ids -> global voxel coordinates."""
    torch = _torch()
    nx, ny, nz = dims
    nbx, nby = (nx + 3) // 4, (ny + 3) // 4
    b = block.to(torch.int64)
    org = torch.stack([b % nbx, (b // nbx) % nby, b // (nbx * nby)], dim=1) * 4
    dt = dtype or xyz.dtype
    return xyz.to(dt) + org.to(dt)


class _Handle:
    _h = None

    def close(self):
        if self._h:
            lib().bcmc_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stats(self):
        st = _capi.Stats()
        _capi.check(lib().bcmc_get_stats(self._h, C.byref(st)))
        return st.as_dict()

    def set_vertex_format(self, fmt):
        """"f32" (16-byte records [n, 4] int32: x, y, z as float32 bits, block),
        "edge8" (8-byte edge records [n] int64, see edge8_positions) or "q10"
        (the paper's 8-byte 10-bit quantised vertices [n] int64, see
        q10_positions)."""
        code = ({"f32": VERTEX_F32, "edge8": VERTEX_EDGE8, "q10": VERTEX_Q10}[fmt]
                if isinstance(fmt, str) else int(fmt))
        _capi.check(lib().bcmc_set_vertex_format(self._h, code))
        self._vfmt = code

    def set_profiling(self, on=True, stages=None):
        """HIP events around every extract stage (on), none (off), or only
        around the stages listed in `stages` (indices into stats()["stage_ms"])."""
        if stages is None:
            _capi.check(lib().bcmc_set_profiling(self._h, 1 if on else 0))
        else:
            mask = 0
            for i in stages:
                mask |= 1 << int(i)
            _capi.check(lib().bcmc_set_profiling_stages(self._h, mask if on else 0))

    def _alloc_out(self, cap):
        torch = _torch()
        if getattr(self, "_vfmt", VERTEX_F32) in (VERTEX_EDGE8, VERTEX_Q10):
            return torch.empty(max(cap, 1), dtype=torch.int64, device="cuda")
        return torch.empty((max(cap, 1), 4), dtype=torch.int32, device="cuda")

    def _records(self, out):
        """Capacity of `out` in records of this volume's format."""
        size = 8 if getattr(self, "_vfmt", VERTEX_F32) in (VERTEX_EDGE8, VERTEX_Q10) else 16
        return out.numel() * out.element_size() // size

    def extract(self, iso, out=None, stream=None):
        """Triangle soup at `iso`: ([3T, 4] int32 CUDA tensor, T).  `out` is
        reused (and grown when too small)."""
        cap = 0 if out is None else self._records(out)
        if out is None:
            out = self._alloc_out(getattr(self, "_cap_hint", 1 << 16))
            cap = self._records(out)
        T = C.c_uint64(0)
        rc = lib().bcmc_extract(self._h, C.c_float(iso), _dev_ptr(out), cap, C.byref(T),
                                _stream_ptr(stream))
        if rc == _capi.E_CAPACITY:
            need = 3 * T.value
            self._cap_hint = need + need // 8 + 1024
            out = self._alloc_out(self._cap_hint)
            rc = lib().bcmc_extract(self._h, C.c_float(iso), _dev_ptr(out), self._records(out),
                                    C.byref(T), _stream_ptr(stream))
        _capi.check(rc)
        self._cap_hint = max(getattr(self, "_cap_hint", 0), 3 * T.value)
        return out[: 3 * T.value], int(T.value)

    def extract_into(self, iso, out, stream=None):
        """Extract into a preallocated buffer ([cap, 4] int32 for "f32"
        records, [cap] int64 for "edge8"); returns (rc, T)."""
        T = C.c_uint64(0)
        rc = lib().bcmc_extract(self._h, C.c_float(iso), _dev_ptr(out), self._records(out),
                                C.byref(T), _stream_ptr(stream))
        return rc, int(T.value)

    # ---- inspection ------------------------------------------------------
    def ranges(self):
        r = np.empty((self.n_blocks, 2), dtype=np.float32)
        _capi.check(lib().bcmc_debug_ranges(self._h, r.ctypes.data_as(C.c_void_p)))
        return r

    def active(self, with_flags=False):
        """(M_active as 0/1 per block, I_active); with_flags adds the per-block
        "can emit" flags of the last extract."""
        a = np.empty(self.n_blocks, dtype=np.uint8)
        ids = np.empty(self.n_blocks, dtype=np.uint32)
        n = C.c_uint64(0)
        _capi.check(lib().bcmc_debug_active(self._h, a.ctypes.data_as(C.c_void_p),
                                            ids.ctypes.data_as(C.c_void_p), C.byref(n)))
        if with_flags:
            return a & 1, ids[: n.value].copy(), (a >> 1) & 1
        return a & 1, ids[: n.value].copy()

    def block_counts(self):
        n = self.stats()["n_active"]
        cnt = np.empty(max(n, 1), dtype=np.uint32)
        off = np.empty(max(n, 1), dtype=np.uint64)
        _capi.check(lib().bcmc_debug_block_counts(self._h, cnt.ctypes.data_as(C.c_void_p),
                                                  off.ctypes.data_as(C.c_void_p), n))
        return cnt[:n], off[:n]

    def cases(self, iso, stream=None):
        torch = _torch()
        n = self.stats()["n_active"]
        d = torch.zeros((max(n, 1), 64), dtype=torch.uint8, device="cuda")
        _capi.check(lib().bcmc_debug_cases(self._h, C.c_float(iso), _dev_ptr(d),
                                           _stream_ptr(stream)))
        return d[:n]


class Volume(_Handle):
    """A fixed-rate ZFP compressed volume resident on the GPU, with its LRU
    block cache (paper Sec. 4)."""

    def __init__(self, stream_words, dims, dtype="f32", rate=8, stream=None):
        torch = _torch()
        nx, ny, nz = (int(d) for d in dims)
        self.dims = (nx, ny, nz)
        self.rate = int(rate)
        self.type = _TYPES[dtype] if isinstance(dtype, str) else int(dtype)
        self.n_blocks = num_blocks(nx, ny, nz)
        h = C.c_void_p()
        if isinstance(stream_words, np.ndarray):
            w = np.ascontiguousarray(stream_words, dtype=np.uint64)
            rc = lib().bcmc_load_compressed(w.ctypes.data_as(C.c_void_p), w.nbytes, 0, nx, ny, nz,
                                            self.type, self.rate, _stream_ptr(stream), C.byref(h))
        else:
            w = stream_words.contiguous()
            dev = 1 if w.is_cuda else 0
            rc = lib().bcmc_load_compressed(C.c_void_p(w.data_ptr()), w.numel() * w.element_size(),
                                            dev, nx, ny, nz, self.type, self.rate,
                                            _stream_ptr(stream), C.byref(h))
        _capi.check(rc)
        self._h = h

    def set_cache_budget(self, initial_bytes=0, max_bytes=0):
        _capi.check(lib().bcmc_set_cache_budget(self._h, int(initial_bytes), int(max_bytes)))

    def reset_cache(self, stream=None):
        _capi.check(lib().bcmc_reset_cache(self._h, _stream_ptr(stream)))

    def decode_all(self, out=None, stream=None):
        """Every block decoded: [N_b, 64] float32 CUDA tensor (into `out`)."""
        torch = _torch()
        if out is None:
            out = torch.empty((self.n_blocks, 64), dtype=torch.float32, device="cuda")
        elif tuple(out.shape) != (self.n_blocks, 64) or out.dtype != torch.float32:
            raise ValueError("out must be a [N_b, 64] float32 CUDA tensor")
        _capi.check(lib().bcmc_decode_all(self._h, _dev_ptr(out), _stream_ptr(stream)))
        return out

    def age_cache(self, k, stream=None):
        """Advance the cache by k calls at which no block is active (test hook)."""
        _capi.check(lib().bcmc_debug_age_cache(self._h, int(k), _stream_ptr(stream)))

    def cache_state(self):
        ns = C.c_uint64(0)
        _capi.check(lib().bcmc_debug_cache_state(self._h, None, None, None, C.byref(ns)))
        n = ns.value
        I_slot = np.empty(self.n_blocks, dtype=np.int32)
        S_block = np.empty(max(n, 1), dtype=np.int32)
        S_age = np.empty(max(n, 1), dtype=np.uint32)
        _capi.check(lib().bcmc_debug_cache_state(
            self._h, I_slot.ctypes.data_as(C.c_void_p), S_block.ctypes.data_as(C.c_void_p),
            S_age.ctypes.data_as(C.c_void_p), C.byref(ns)))
        return I_slot, S_block[:n], S_age[:n]

    def slot_data(self):
        n = self.stats()["n_slots"]
        out = np.empty((max(n, 1), 64), dtype=np.float32)
        _capi.check(lib().bcmc_debug_slot_data(self._h, out.ctypes.data_as(C.c_void_p)))
        return out[:n]

    def new_blocks(self):
        ids = np.empty(self.n_blocks, dtype=np.uint32)
        n = C.c_uint64(0)
        _capi.check(lib().bcmc_debug_new(self._h, ids.ctypes.data_as(C.c_void_p), C.byref(n)))
        return ids[: n.value].copy()


class FieldVolume(_Handle):
    """A volume over decoded float blocks ([N_b, 64] CUDA float32 tensor, kept
    referenced here): all blocks resident, no cache.  Differentiable."""

    def __init__(self, blocks, dims, stream=None):
        nx, ny, nz = (int(d) for d in dims)
        self.dims = (nx, ny, nz)
        self.n_blocks = num_blocks(nx, ny, nz)
        if tuple(blocks.shape) != (self.n_blocks, 64) or not blocks.is_cuda:
            raise ValueError("blocks must be a CUDA tensor of shape [N_b, 64]")
        self.blocks = blocks.contiguous()
        h = C.c_void_p()
        _capi.check(lib().bcmc_volume_from_blocks(_dev_ptr(self.blocks), nx, ny, nz,
                                                  _stream_ptr(stream), C.byref(h)))
        self._h = h

    def rebind(self, blocks, stream=None):
        """Use new decoded blocks (same dims); ranges are recomputed on the GPU."""
        if tuple(blocks.shape) != (self.n_blocks, 64) or not blocks.is_cuda:
            raise ValueError("blocks must be a CUDA tensor of shape [N_b, 64]")
        self.blocks = blocks.contiguous()
        _capi.check(lib().bcmc_rebind_blocks(self._h, _dev_ptr(self.blocks), _stream_ptr(stream)))

    def backward(self, iso, gV, stream=None):
        torch = _torch()
        gV = gV.contiguous().to(torch.float32)
        dfield = torch.empty((self.n_blocks, 64), dtype=torch.float32, device="cuda")
        diso = torch.empty((), dtype=torch.float32, device="cuda")
        n = gV.shape[0]
        _capi.check(lib().bcmc_backward(self._h, C.c_float(iso),
                                        _dev_ptr(gV) if n else None, n, _dev_ptr(dfield),
                                        _dev_ptr(diso), _stream_ptr(stream)))
        return dfield, diso


class Batch:
    """Many volumes x isovalues extracted in one persistent launch (hipGraph
    replay).  jobs: list of (volume_index, isovalue)."""

    def __init__(self, volumes, jobs, stream=None):
        self.volumes = list(volumes)       # keep the volumes alive
        self.n_jobs = len(jobs)
        jv = np.ascontiguousarray([j[0] for j in jobs], dtype=np.uint32)
        ji = np.ascontiguousarray([j[1] for j in jobs], dtype=np.float32)
        arr = (C.c_void_p * len(self.volumes))(*[v._h for v in self.volumes])
        h = C.c_void_p()
        _capi.check(lib().bcmc_batch_create(arr, len(self.volumes), jv.ctypes.data_as(C.c_void_p),
                                            ji.ctypes.data_as(C.c_void_p), self.n_jobs,
                                            _stream_ptr(stream), C.byref(h)))
        self._h = h
        self._out = None

    def close(self):
        if getattr(self, "_h", None):
            lib().bcmc_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_isos(self, isos, stream=None):
        a = np.ascontiguousarray(isos, dtype=np.float32)
        assert a.shape == (self.n_jobs,)
        _capi.check(lib().bcmc_batch_set_isos(self._h, a.ctypes.data_as(C.c_void_p), _stream_ptr(stream)))

    def reset(self, stream=None):
        _capi.check(lib().bcmc_batch_reset(self._h, _stream_ptr(stream)))

    def set_graph(self, on=True):
        _capi.check(lib().bcmc_batch_set_graph(self._h, 1 if on else 0))

    def set_schedule(self, stage_blocks, per_cu, front_per_cu, scan=0):
        _capi.check(lib().bcmc_batch_set_schedule(self._h, int(stage_blocks), int(per_cu),
                                                  int(front_per_cu), int(scan)))

    def tune(self, cache_path=None, stream=None):
        _capi.check(lib().bcmc_batch_tune(self._h, cache_path.encode() if cache_path else None,
                                          _stream_ptr(stream)))

    def info(self):
        st = _capi.BatchInfo()
        _capi.check(lib().bcmc_batch_get_info(self._h, C.byref(st)))
        return st.as_dict()

    def run_into(self, out, stream=None):
        """Run into a preallocated [cap, 4] int32 buffer: (rc, job offsets [n_jobs+1])."""
        offs = np.zeros(self.n_jobs + 1, dtype=np.uint64)
        rc = lib().bcmc_batch_run(self._h, _dev_ptr(out), out.shape[0],
                                  offs.ctypes.data_as(C.c_void_p), _stream_ptr(stream))
        return rc, offs

    def run(self, stream=None):
        """(vertices [V, 4] int32 CUDA tensor of all jobs, job offsets)."""
        torch = _torch()
        if self._out is None:
            self._out = torch.empty((1 << 16, 4), dtype=torch.int32, device="cuda")
        rc, offs = self.run_into(self._out, stream)
        if rc == _capi.E_CAPACITY:
            need = int(offs[-1])
            self._out = torch.empty((need + need // 8 + 1024, 4), dtype=torch.int32, device="cuda")
            rc, offs = self.run_into(self._out, stream)
        _capi.check(rc)
        return self._out[: int(offs[-1])], offs


class DenseMC:
    """The dense data-parallel marching cubes baseline (Sec. 3.3.3) over an
    uncompressed [nz, ny, nx] float32 CUDA field: the same 16-byte records
    as Volume.extract, cells in global row-major order."""

    def __init__(self, dims):
        nx, ny, nz = (int(d) for d in dims)
        self.dims = (nx, ny, nz)
        h = C.c_void_p()
        _capi.check(lib().bcmc_dense_create(nx, ny, nz, C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().bcmc_dense_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def extract_into(self, field, iso, out, stream=None):
        """Into a preallocated [cap, 4] int32 buffer: (rc, T)."""
        nx, ny, nz = self.dims
        if tuple(field.shape) != (nz, ny, nx) or not field.is_cuda or not field.is_contiguous():
            raise ValueError("field must be a contiguous [nz, ny, nx] CUDA tensor")
        T = C.c_uint64(0)
        rc = lib().bcmc_dense_extract(self._h, _dev_ptr(field), C.c_float(iso),
                                      _dev_ptr(out) if out.shape[0] else None, out.shape[0],
                                      C.byref(T), _stream_ptr(stream))
        if rc not in (_capi.OK, _capi.E_CAPACITY):
            _capi.check(rc)
        return rc, int(T.value)

    def extract(self, field, iso, stream=None):
        """([3T, 4] int32 CUDA tensor, T)."""
        torch = _torch()
        out = torch.empty((1, 4), dtype=torch.int32, device="cuda")
        rc, T = self.extract_into(field, iso, out, stream)
        if rc == _capi.E_CAPACITY:
            out = torch.empty((3 * T + 16, 4), dtype=torch.int32, device="cuda")
            rc, T = self.extract_into(field, iso, out, stream)
        _capi.check(rc)
        return out[: 3 * T], T

    def active_cells(self):
        n = C.c_uint64(0)
        _capi.check(lib().bcmc_dense_active_cells(self._h, C.byref(n)))
        return int(n.value)


def extract_blocks_noalloc(blocks, dims, iso, out, stream=None):
    """Extraction over decoded blocks ([N_b, 64] CUDA float32) into a
    preallocated [cap, 4] int32 CUDA tensor without any device allocation
    (every scratch buffer lives in the library's static array of about 2^19
    blocks).  Returns (rc, T); rc is 0 or an error code (E_CAPACITY: T is set,
    enlarge `out` and call again)."""
    nx, ny, nz = (int(d) for d in dims)
    if tuple(blocks.shape) != (num_blocks(nx, ny, nz), 64) or not blocks.is_cuda:
        raise ValueError("blocks must be a CUDA tensor of shape [N_b, 64]")
    if not blocks.is_contiguous() or not out.is_contiguous():
        raise ValueError("blocks and out must be contiguous")
    T = C.c_uint64(0)
    rc = lib().bcmc_extract_blocks_noalloc(_dev_ptr(blocks), nx, ny, nz, C.c_float(iso),
                                           _dev_ptr(out) if out.shape[0] else None, out.shape[0],
                                           C.byref(T), _stream_ptr(stream))
    if rc not in (_capi.OK, _capi.E_CAPACITY):
        _capi.check(rc)
    return rc, int(T.value)


_POOL = {}


def _acquire_field_volume(blocks, dims):
    """A FieldVolume for `dims` bound to `blocks`, reused across calls (a
    handle holds the state of one forward until its backward is done)."""
    free = _POOL.setdefault(tuple(dims), [])
    if free:
        vol = free.pop()
        vol.rebind(blocks)
        return vol
    return FieldVolume(blocks, dims)


def _release_field_volume(vol):
    _POOL.setdefault(vol.dims, []).append(vol)


def _make_extract_fn():
    torch = _torch()

    class ExtractFn(torch.autograd.Function):
        """verts_xyz, vblock = ExtractFn.apply(field_blocks, iso, dims).

        field_blocks: [N_b, 64] float32 CUDA tensor (block layout); iso: 0-d
        float tensor.  Returns block-relative vertex positions [3T, 3]
        (differentiable) and block ids [3T] (int32).  Gradients flow to
        field_blocks and iso through t = (iso - a)/(b - a), topology fixed."""

        @staticmethod
        def forward(ctx, field_blocks, iso, dims, keep=True):
            # keep: a backward may follow, so the volume (which holds this
            # extract's layout) stays with ctx until then; otherwise it goes
            # straight back to the pool.  The soup is a fresh buffer: its
            # views are returned without a copy.
            vol = _acquire_field_volume(field_blocks.detach(), dims)
            # the isovalue is a kernel argument, read on the host; the extract
            # reads its triangle count back anyway, so the forward synchronises
            # with the stream once in any case
            isof = float(iso)
            verts, T = vol.extract(isof)
            xyz, blk = split_vertices(verts)
            ctx.iso = isof
            ctx.iso_dtype = iso.dtype if torch.is_tensor(iso) else torch.float32
            if keep:
                # autograd's version counter then rejects an in-place edit of
                # the field between this forward and its backward
                ctx.save_for_backward(field_blocks)
                ctx.vol = vol
            else:
                ctx.vol = None
                _release_field_volume(vol)
            ctx.mark_non_differentiable(blk)
            return xyz, blk

        @staticmethod
        def backward(ctx, g_xyz, g_blk):
            if ctx.vol is None:
                raise RuntimeError("ExtractFn: backward of a forward run without gradients")
            vol, ctx.vol = ctx.vol, None
            try:
                ctx.saved_tensors          # raises if the field was modified in place
                dfield, diso = vol.backward(ctx.iso, g_xyz)
            finally:
                _release_field_volume(vol)
            return dfield, diso.to(ctx.iso_dtype), None, None

    return ExtractFn


class _LazyFn:
    _fn = None

    def _get(self):
        if _LazyFn._fn is None:
            _LazyFn._fn = _make_extract_fn()
        return _LazyFn._fn

    def apply(self, field_blocks, iso, dims):
        torch = _torch()
        keep = torch.is_grad_enabled() and (
            field_blocks.requires_grad or (torch.is_tensor(iso) and iso.requires_grad))
        return self._get().apply(field_blocks, iso, dims, keep)

    def __getattr__(self, name):
        return getattr(self._get(), name)


ExtractFn = _LazyFn()
