"""CPU oracle (TEST INFRASTRUCTURE ONLY).

Thin ctypes binding of ``oracle/oracle.c``: a plain single-threaded C
implementation of what the block-compressed isosurface path computes.  Only
the tests, the smoke check and the benchmark's CPU-baseline leg may load it;
the product library never does, and the two share no code.

``build()`` compiles ``liboracle.so`` with gcc (-O2 -ffp-contract=off, no
fast-math).  Functions not covered by an independent pin are marked
"parity unpinned" in ``oracle.c``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-Wall",
          "-Wextra", "-shared", "-fPIC"]


def build(force=True):
    """Compile liboracle.so from oracle.c (always, unless force=False and the
    library is newer than its source)."""
    if (not force and os.path.exists(LIB)
            and os.path.getmtime(LIB) >= os.path.getmtime(SRC)):
        return LIB
    tmp = LIB + ".tmp"
    subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"])
    os.replace(tmp, LIB)
    return LIB


_lib = None
_P = C.c_void_p
_u32, _u64, _i32, _f32, _f64, _int = C.c_uint32, C.c_uint64, C.c_int32, C.c_float, C.c_double, C.c_int


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        sig = {
            "oracle_num_blocks": (_u64, [_u32, _u32, _u32]),
            "oracle_zfp_encode": (_int, [_P, _int, _u32, _u32, _u32, _u32, _P]),
            "oracle_zfp_decode": (_int, [_P, _int, _u32, _u32, _u32, _u32, _P]),
            "oracle_zfp_decode_f64": (_int, [_P, _u32, _u32, _u32, _u32, _P]),
            "oracle_zfp_decode_some": (_int, [_P, _int, _u32, _P, _u64, _P]),
            "oracle_fwd_lift": (None, [_P, _int]),
            "oracle_inv_lift": (None, [_P, _int]),
            "oracle_sequency_order": (None, [_P]),
            "oracle_to_negabinary": (_u64, [C.c_int64, _int]),
            "oracle_from_negabinary": (C.c_int64, [_u64, _int]),
            "oracle_encode_planes": (_u64, [_P, _int, _u64, _P]),
            "oracle_decode_planes": (None, [_P, _int, _u64, _P]),
            "oracle_block_ranges": (None, [_P, _u32, _u32, _u32, _P]),
            "oracle_active_blocks": (_u64, [_P, _u32, _u32, _u32, _f32, _P]),
            "oracle_mc_tables": (None, [_P, _P, _P]),
            "oracle_mc_extract": (_u64, [_P, _u32, _u32, _u32, _f32, _P, _P, _P, _P, _P, _P]),
            "oracle_mc_extract_f32": (_u64, [_P, _u32, _u32, _u32, _f32, _P, _P]),
            "oracle_mc_extract_edge8": (_u64, [_P, _u32, _u32, _u32, _f32, _P]),
            "oracle_mc_extract_q10": (_u64, [_P, _u32, _u32, _u32, _f32, _P]),
            "oracle_brute_count": (_u64, [_P, _u32, _u32, _u32, _f32]),
            "oracle_mc_extract_dense": (_u64, [_P, _u32, _u32, _u32, _f32, _P, _P]),
            "oracle_brute_count_blocks": (_u64, [_P, _u32, _u32, _u32, _f32]),
            "oracle_block_vertex_counts": (None, [_P, _u32, _u32, _u32, _f32, _P, _u64, _P]),
            "oracle_lru_create": (_P, [_u64, _u64, _u64]),
            "oracle_lru_free": (None, [_P]),
            "oracle_lru_update": (_int, [_P, _P, _P, _P, _P]),
            "oracle_lru_n_slots": (_u64, [_P]),
            "oracle_lru_idle": (None, [_P, _u64]),
            "oracle_lru_state": (None, [_P, _P, _P, _P]),
            "oracle_sphere_loss": (_f64, [_P, _u64, _P, _f64, _P]),
            "oracle_mc_backward": (None, [_P, _u32, _u32, _u32, _f32, _P, _P, _P]),
            "oracle_sphere_loss_fixed_topology": (
                _f64, [_P, _P, _u32, _u32, _u32, _f32, _f64, _P, _f64]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def num_blocks(nx, ny, nz):
    return int(lib().oracle_num_blocks(nx, ny, nz))


def block_dims(nx, ny, nz):
    return ((nx + 3) // 4, (ny + 3) // 4, (nz + 3) // 4)


# ---- ZFP -----------------------------------------------------------------

def zfp_encode(field, rate):
    """Fixed-rate encode of a [nz][ny][nx] float32/float64 array -> u64 words."""
    field = np.ascontiguousarray(field)
    is_f64 = 1 if field.dtype == np.float64 else 0
    if field.dtype not in (np.float32, np.float64):
        raise TypeError("field must be float32 or float64")
    nz, ny, nx = field.shape
    out = np.zeros(num_blocks(nx, ny, nz) * rate, dtype=np.uint64)
    rc = lib().oracle_zfp_encode(_ptr(field), is_f64, nx, ny, nz, rate, _ptr(out))
    if rc != 0:
        raise ValueError(f"oracle_zfp_encode failed ({rc})")
    return out


def zfp_decode(stream, dims, rate, is_f64=False):
    """Decode every block -> float32 [N_b, 64] (block layout)."""
    nx, ny, nz = dims
    stream = np.ascontiguousarray(stream, dtype=np.uint64)
    out = np.empty((num_blocks(nx, ny, nz), 64), dtype=np.float32)
    rc = lib().oracle_zfp_decode(_ptr(stream), int(is_f64), nx, ny, nz, rate, _ptr(out))
    if rc != 0:
        raise ValueError(f"oracle_zfp_decode failed ({rc})")
    return out


def zfp_decode_f64(stream, dims, rate):
    nx, ny, nz = dims
    stream = np.ascontiguousarray(stream, dtype=np.uint64)
    out = np.empty((num_blocks(nx, ny, nz), 64), dtype=np.float64)
    rc = lib().oracle_zfp_decode_f64(_ptr(stream), nx, ny, nz, rate, _ptr(out))
    if rc != 0:
        raise ValueError(f"oracle_zfp_decode_f64 failed ({rc})")
    return out


def zfp_decode_some(stream, ids, rate, is_f64=False):
    stream = np.ascontiguousarray(stream, dtype=np.uint64)
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    out = np.empty((len(ids), 64), dtype=np.float32)
    rc = lib().oracle_zfp_decode_some(_ptr(stream), int(is_f64), rate, _ptr(ids), len(ids), _ptr(out))
    if rc != 0:
        raise ValueError("oracle_zfp_decode_some failed")
    return out


def fwd_lift(v, is_f64=False):
    a = np.array(v, dtype=np.int64)
    lib().oracle_fwd_lift(_ptr(a), int(is_f64))
    return a


def inv_lift(v, is_f64=False):
    a = np.array(v, dtype=np.int64)
    lib().oracle_inv_lift(_ptr(a), int(is_f64))
    return a


def sequency_order():
    p = np.zeros(64, dtype=np.int32)
    lib().oracle_sequency_order(_ptr(p))
    return p


def to_negabinary(i, is_f64=False):
    return int(lib().oracle_to_negabinary(int(i), int(is_f64)))


def from_negabinary(u, is_f64=False):
    return int(lib().oracle_from_negabinary(int(u), int(is_f64)))


def encode_planes(u, maxbits, is_f64=False):
    u = np.ascontiguousarray(u, dtype=np.uint64)
    words = np.zeros(maxbits // 64 + 2, dtype=np.uint64)
    used = lib().oracle_encode_planes(_ptr(u), int(is_f64), maxbits, _ptr(words))
    return words, int(used)


def decode_planes(words, maxbits, is_f64=False):
    words = np.ascontiguousarray(words, dtype=np.uint64)
    u = np.zeros(64, dtype=np.uint64)
    lib().oracle_decode_planes(_ptr(words), int(is_f64), maxbits, _ptr(u))
    return u


# ---- blocks <-> dense ----------------------------------------------------

def field_to_blocks(field):
    """Dense [nz][ny][nx] -> [N_b, 64] block layout, padded by replication."""
    nz, ny, nx = field.shape
    nbx, nby, nbz = block_dims(nx, ny, nz)
    p = np.pad(field, ((0, 4 * nbz - nz), (0, 4 * nby - ny), (0, 4 * nbx - nx)), mode="edge")
    p = p.reshape(nbz, 4, nby, 4, nbx, 4).transpose(0, 2, 4, 1, 3, 5)
    return np.ascontiguousarray(p.reshape(-1, 64))


def blocks_to_field(blocks, dims):
    nx, ny, nz = dims
    nbx, nby, nbz = block_dims(nx, ny, nz)
    p = np.asarray(blocks).reshape(nbz, nby, nbx, 4, 4, 4).transpose(0, 3, 1, 4, 2, 5)
    return np.ascontiguousarray(p.reshape(4 * nbz, 4 * nby, 4 * nbx)[:nz, :ny, :nx])


# ---- ranges / culling ----------------------------------------------------

def block_ranges(blocks, dims):
    nx, ny, nz = dims
    blocks = np.ascontiguousarray(blocks, dtype=np.float32)
    out = np.empty((num_blocks(nx, ny, nz), 2), dtype=np.float32)
    lib().oracle_block_ranges(_ptr(blocks), nx, ny, nz, _ptr(out))
    return out


def active_blocks(ranges, dims, iso):
    nx, ny, nz = dims
    ranges = np.ascontiguousarray(ranges, dtype=np.float32)
    out = np.empty(num_blocks(nx, ny, nz), dtype=np.uint8)
    lib().oracle_active_blocks(_ptr(ranges), nx, ny, nz, float(iso), _ptr(out))
    return out


# ---- marching cubes ------------------------------------------------------

def mc_tables():
    nt = np.zeros(256, dtype=np.int32)
    tri = np.zeros((256, 16), dtype=np.int32)
    em = np.zeros(256, dtype=np.int32)
    lib().oracle_mc_tables(_ptr(nt), _ptr(tri), _ptr(em))
    return nt, tri, em


def mc_extract(blocks, dims, iso, want=("verts", "vblock")):
    """Plain MC over the whole decoded field, canonical order.

    Returns a dict with the requested arrays among verts (float64 [3T,3],
    block-local), vblock (uint32 [3T]), vedge (int64 [3T]), cell_keys
    (uint64 [n_cells]), cases (uint8 [n_cells]) plus T and n_cells."""
    nx, ny, nz = dims
    blocks = np.ascontiguousarray(blocks, dtype=np.float32)
    L = lib()
    nc = C.c_uint64(0)
    T = int(L.oracle_mc_extract(_ptr(blocks), nx, ny, nz, float(iso), None, None, None,
                                None, None, C.byref(nc)))
    n_cells = int(nc.value)
    out = {"T": T, "n_cells": n_cells}
    arrs = {
        "verts": np.empty((3 * T, 3), dtype=np.float64) if "verts" in want else None,
        "vblock": np.empty(3 * T, dtype=np.uint32) if "vblock" in want else None,
        "vedge": np.empty(3 * T, dtype=np.int64) if "vedge" in want else None,
        "cell_keys": np.empty(n_cells, dtype=np.uint64) if "cell_keys" in want else None,
        "cases": np.empty(n_cells, dtype=np.uint8) if "cases" in want else None,
    }
    if any(a is not None for a in arrs.values()):
        T2 = L.oracle_mc_extract(_ptr(blocks), nx, ny, nz, float(iso), _ptr(arrs["verts"]),
                                 _ptr(arrs["vblock"]), _ptr(arrs["vedge"]),
                                 _ptr(arrs["cell_keys"]), _ptr(arrs["cases"]), None)
        assert T2 == T
    for k, v in arrs.items():
        if v is not None:
            out[k] = v
    return out


def mc_extract_f32(blocks, dims, iso):
    nx, ny, nz = dims
    blocks = np.ascontiguousarray(blocks, dtype=np.float32)
    T = mc_count(blocks, dims, iso)
    v = np.empty((3 * T, 3), dtype=np.float32)
    vb = np.empty(3 * T, dtype=np.uint32)
    lib().oracle_mc_extract_f32(_ptr(blocks), nx, ny, nz, float(iso), _ptr(v), _ptr(vb))
    return v, vb


def mc_extract_edge8(blocks, dims, iso):
    """The canonical soup as 64-bit edge records (block | cell << 32 |
    edge << 38 | q << 42, q = min(trunc(t * 2^22), 2^22 - 1), t in float32)."""
    nx, ny, nz = dims
    blocks = np.ascontiguousarray(blocks, dtype=np.float32)
    T = mc_count(blocks, dims, iso)
    rec = np.empty(max(3 * T, 1), dtype=np.uint64)
    lib().oracle_mc_extract_edge8(_ptr(blocks), nx, ny, nz, float(iso), _ptr(rec))
    return rec[: 3 * T]


def mc_extract_q10(blocks, dims, iso):
    """The canonical soup as Sec. 4.5's 8-byte vertices: 10-bit block-relative
    coordinates x | y << 10 | z << 20 (low 32 bits), block id (high 32)."""
    nx, ny, nz = dims
    blocks = np.ascontiguousarray(blocks, dtype=np.float32)
    T = mc_count(blocks, dims, iso)
    rec = np.empty(max(3 * T, 1), dtype=np.uint64)
    lib().oracle_mc_extract_q10(_ptr(blocks), nx, ny, nz, float(iso), _ptr(rec))
    return rec[: 3 * T]


def q10_positions(records):
    """Block-relative float64 positions q * 4 / 1023 of Sec. 4.5's 8-byte
    vertices, with their block ids."""
    r = np.asarray(records, dtype=np.uint64)
    code = (r & np.uint64(0xFFFFFFFF)).astype(np.int64)
    block = (r >> np.uint64(32)).astype(np.uint32)
    q = np.stack([code & 1023, (code >> 10) & 1023, (code >> 20) & 1023], axis=1)
    return q.astype(np.float64) * (4.0 / 1023.0), block


def edge8_positions(records):
    """Block-relative float64 positions of 64-bit edge records: the edge's
    first corner plus (q + 0.5) / 2^22 along its axis; with the block ids."""
    r = np.asarray(records, dtype=np.uint64)
    block = (r & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    cell = ((r >> np.uint64(32)) & np.uint64(63)).astype(np.int64)
    e = ((r >> np.uint64(38)) & np.uint64(15)).astype(np.int64)
    q = (r >> np.uint64(42)).astype(np.float64)
    axis = e >> 2
    b0, b1 = e & 1, (e >> 1) & 1
    off = np.zeros((len(r), 3), dtype=np.int64)
    off[:, 0] = np.where(axis == 0, 0, b0)
    off[:, 1] = np.where(axis == 1, 0, np.where(axis == 0, b0, b1))
    off[:, 2] = np.where(axis == 2, 0, b1)
    pos = np.stack([cell & 3, (cell >> 2) & 3, cell >> 4], axis=1) + off
    pos = pos.astype(np.float64)
    pos[np.arange(len(r)), axis] += (q + 0.5) / 4194304.0
    return pos, block


def mc_count(blocks, dims, iso):
    nx, ny, nz = dims
    blocks = np.ascontiguousarray(blocks, dtype=np.float32)
    return int(lib().oracle_mc_extract(_ptr(blocks), nx, ny, nz, float(iso), None, None,
                                       None, None, None, None))


def mc_extract_dense(field, iso):
    """Plain MC over a dense [nz][ny][nx] field, cells in global z, y, x
    order: (float32 block-relative vertices [3T, 3], block ids [3T])."""
    field = np.ascontiguousarray(field, dtype=np.float32)
    nz, ny, nx = field.shape
    T = int(lib().oracle_mc_extract_dense(_ptr(field), nx, ny, nz, float(iso), None, None))
    v = np.empty((max(3 * T, 1), 3), dtype=np.float32)
    vb = np.empty(max(3 * T, 1), dtype=np.uint32)
    lib().oracle_mc_extract_dense(_ptr(field), nx, ny, nz, float(iso), _ptr(v), _ptr(vb))
    return v[: 3 * T], vb[: 3 * T]


def brute_count(field, iso):
    field = np.ascontiguousarray(field, dtype=np.float32)
    nz, ny, nx = field.shape
    return int(lib().oracle_brute_count(_ptr(field), nx, ny, nz, float(iso)))


def brute_count_blocks(blocks, dims, iso):
    nx, ny, nz = dims
    blocks = np.ascontiguousarray(blocks, dtype=np.float32)
    return int(lib().oracle_brute_count_blocks(_ptr(blocks), nx, ny, nz, float(iso)))


def block_vertex_counts(blocks, dims, iso, ids):
    nx, ny, nz = dims
    blocks = np.ascontiguousarray(blocks, dtype=np.float32)
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    out = np.empty(len(ids), dtype=np.uint32)
    lib().oracle_block_vertex_counts(_ptr(blocks), nx, ny, nz, float(iso), _ptr(ids),
                                     len(ids), _ptr(out))
    return out


# ---- LRU cache (Alg. 1) --------------------------------------------------

class LRU:
    """Serial simulator of the GPU-driven LRU block cache (Sec. 4.2, Alg. 1)."""

    def __init__(self, n_blocks, initial_slots, max_slots):
        self.n_blocks = int(n_blocks)
        self._h = lib().oracle_lru_create(n_blocks, initial_slots, max_slots)

    def __del__(self):
        if getattr(self, "_h", None):
            lib().oracle_lru_free(self._h)
            self._h = None

    def update(self, active):
        active = np.ascontiguousarray(active, dtype=np.uint8)
        assert active.shape == (self.n_blocks,)
        I_new = np.empty(self.n_blocks, dtype=np.uint32)
        n_new = C.c_uint64(0)
        n_ev = C.c_uint64(0)
        rc = lib().oracle_lru_update(self._h, _ptr(active), _ptr(I_new), C.byref(n_new),
                                     C.byref(n_ev))
        return rc, I_new[: n_new.value].copy(), int(n_ev.value)

    def idle(self, k):
        """k updates at which no block is active, at once."""
        lib().oracle_lru_idle(self._h, int(k))

    @property
    def n_slots(self):
        return int(lib().oracle_lru_n_slots(self._h))

    def state(self):
        ns = self.n_slots
        I_slot = np.empty(self.n_blocks, dtype=np.int32)
        S_block = np.empty(max(ns, 1), dtype=np.int32)
        S_age = np.empty(max(ns, 1), dtype=np.uint32)
        lib().oracle_lru_state(self._h, _ptr(I_slot), _ptr(S_block), _ptr(S_age))
        return I_slot, S_block[:ns], S_age[:ns]


# ---- gradient ------------------------------------------------------------

def sphere_loss(verts_global, center, radius):
    v = np.ascontiguousarray(verts_global, dtype=np.float64)
    c = np.ascontiguousarray(center, dtype=np.float64)
    g = np.empty_like(v)
    L = lib().oracle_sphere_loss(_ptr(v), len(v), _ptr(c), float(radius), _ptr(g))
    return float(L), g


def mc_backward(blocks, dims, iso, gV):
    nx, ny, nz = dims
    blocks = np.ascontiguousarray(blocks, dtype=np.float32)
    gV = np.ascontiguousarray(gV, dtype=np.float64)
    df = np.empty((num_blocks(nx, ny, nz), 64), dtype=np.float64)
    di = C.c_double(0)
    lib().oracle_mc_backward(_ptr(blocks), nx, ny, nz, float(iso), _ptr(gV), _ptr(df),
                             C.byref(di))
    return df, float(di.value)


def sphere_loss_fixed_topology(field_blocks_f64, blocks_case, dims, iso_case, iso,
                               center, radius):
    nx, ny, nz = dims
    fd = np.ascontiguousarray(field_blocks_f64, dtype=np.float64)
    bc = np.ascontiguousarray(blocks_case, dtype=np.float32)
    c = np.ascontiguousarray(center, dtype=np.float64)
    return float(lib().oracle_sphere_loss_fixed_topology(
        _ptr(fd), _ptr(bc), nx, ny, nz, float(iso_case), float(iso), _ptr(c), float(radius)))


def verts_global(verts_local, vblock, dims):
    """Block-local vertex positions -> global voxel coordinates (float64)."""
    nx, ny, nz = dims
    nbx, nby, _ = block_dims(nx, ny, nz)
    vb = np.asarray(vblock, dtype=np.int64)
    org = np.stack([vb % nbx, (vb // nbx) % nby, vb // (nbx * nby)], axis=1) * 4
    return np.asarray(verts_local, dtype=np.float64) + org
