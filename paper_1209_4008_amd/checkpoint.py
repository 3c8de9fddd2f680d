"""Checkpoints of a gauge field and of the run state that goes with it.

A checkpoint is one .npz file (numpy's zip of plain arrays, read back with
allow_pickle=False) with two members:

  links   float64 array of 72 V reals: the canonical complex128 field
          U[t][z][y][x][mu][a][b] as interleaved (re, im) pairs, the form
          gf_pack reads and gf_unpack writes, whatever the device field's
          precision and storage;
  header  a JSON string: format version, extents, the device field's
          precision and storage, and the caller's run state (gauge, seed,
          the next sweep index, theta history, ... as keyword arguments).

The device field is written through gf_unpack and restored through gf_pack.
Both are exact for every precision and storage: FP32 values and the two
stored rows of a 12-real link convert to FP64 and back unchanged. A run
stopped after sweep k and restored therefore continues bit for bit as if it
had not stopped; annealing resumes exactly because its draws are keyed by
(seed, sweep index, site, subgroup) and not by a generator state.
"""
import json

import numpy as np

from . import FP32, FP64, R12, R18, GFError, ERR_ARG, Geom, field_bytes

FORMAT = 1
_PREC = {FP32: "fp32", FP64: "fp64"}
_STORAGE = {R12: "r12", R18: "r18"}


def write(path, links, dims, prec, storage, state=None):
    """Write canonical links (float64, 72 V reals) and the header to path."""
    dims = [int(v) for v in dims]
    links = np.ascontiguousarray(links, dtype=np.float64).reshape(-1)
    V = int(np.prod(dims))
    if links.size != 72 * V:
        raise GFError(ERR_ARG, f"checkpoint: {links.size} reals for extents {dims}")
    if prec not in _PREC or storage not in _STORAGE:
        raise GFError(ERR_ARG, "checkpoint: bad precision or storage")
    header = {"format": FORMAT, "dims": dims, "precision": _PREC[prec],
              "storage": _STORAGE[storage], "state": dict(state or {})}
    with open(path, "wb") as fh:
        np.savez(fh, links=links, header=np.array(json.dumps(header)))


def read(path):
    """(links, header) of a checkpoint file; links as float64, 72 V reals."""
    with np.load(path, allow_pickle=False) as z:
        if set(z.files) != {"links", "header"}:
            raise GFError(ERR_ARG, f"checkpoint: unexpected members {sorted(z.files)}")
        header = json.loads(str(z["header"]))
        links = np.array(z["links"], dtype=np.float64)
    if header.get("format") != FORMAT:
        raise GFError(ERR_ARG, f"checkpoint: format {header.get('format')} is not {FORMAT}")
    if links.size != 72 * int(np.prod(header["dims"])):
        raise GFError(ERR_ARG, "checkpoint: link count does not match the extents")
    return links, header


def geom_of(header):
    prec = {v: k for k, v in _PREC.items()}[header["precision"]]
    storage = {v: k for k, v in _STORAGE.items()}[header["storage"]]
    return Geom.make(header["dims"], prec, storage)


def save(ctx, path, U, geom, **state):
    """Write the device field U (geometry geom) and the run state to path."""
    torch = ctx.torch
    canon = torch.empty(geom.volume * 72, dtype=torch.float64, device=ctx.stream.device)
    ctx.unpack(geom, U, canon)
    ctx.stream.synchronize()
    write(path, canon.cpu().numpy(), geom.dims, geom.prec, geom.storage, state)


def load(ctx, path, U=None):
    """Restore a checkpoint: (U, geom, state). U, if given, must be a device
    buffer of at least gf_field_bytes(geom); else one is allocated."""
    torch = ctx.torch
    links, header = read(path)
    geom = geom_of(header)
    if U is None:
        U = ctx.empty_field(geom)
    elif U.numel() * U.element_size() < field_bytes(geom):
        raise GFError(ERR_ARG, "checkpoint: the buffer is smaller than the field")
    canon = torch.from_numpy(links).to(ctx.stream.device)
    torch.cuda.current_stream(ctx.stream.device).synchronize()
    ctx.pack(geom, canon, U)
    ctx.stream.synchronize()
    return U, geom, header["state"]
