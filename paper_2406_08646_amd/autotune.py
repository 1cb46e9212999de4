"""Launch-shape autotuners: the batched solver's launch form and shape, and
the tile height of the staged 16-column SpMM.

The batched Jacobi-CG (``spx_batch_cg``) has two launch forms: one launch
per CG phase for the whole batch, or one persistent launch in which each
workgroup solves whole systems from a queue (``persistent``).  The first has
three shape knobs: the number of workgroups shared by the systems, the row
walk (``rows_per_tile`` 0: the library's choice, the window walk when every
system has a window index; 64 or 256: the stream walk with that tile) and
the exponent that turns a system's size into its share of the workgroups.
The best values depend on the mix of system sizes, so the tuner times whole
solves of the actual batch for a small grid of candidates, on the GPU, and
keeps the fastest.  Results are cached per (device, batch signature,
tolerance) in memory and, optionally, in a JSON file.
"""
from __future__ import annotations

import hashlib
import itertools
import json
import os
import time
from dataclasses import asdict, dataclass
from typing import Dict, Iterable, List, Optional

import torch

from . import spx

_MEMO: Dict[str, dict] = {}


@dataclass
class Candidate:
    blocks: int
    rows_per_tile: int
    weight_exponent: float
    persistent: int = -1  # 1: the persistent form (the other knobs unused)


def default_candidates(cus: int) -> List[Candidate]:
    out = [Candidate(0, 0, 1.0, persistent=1)]
    for blocks, rows, gamma in itertools.product((4 * cus, 8 * cus, 16 * cus), (0, 64, 256),
                                                 (0.75, 1.0, 1.25)):
        out.append(Candidate(blocks, rows, gamma))
    return out


def batch_signature(batch: "spx.Batch", rtol: float) -> str:
    h = hashlib.sha1()
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    h.update(f"{props.name}|{getattr(props, 'gcnArchName', '')}|{rtol:.3e}".encode())
    for m in batch.mats:
        h.update(f"{m.n}:{m.nnz};".encode())
    return h.hexdigest()


def tune_batch(batch: "spx.Batch", b: torch.Tensor, rtol: float = 1e-8, maxit: int = 100000,
               candidates: Optional[Iterable[Candidate]] = None, repeats: int = 1,
               cache_file: Optional[str] = None, verbose: bool = False) -> dict:
    """Times full batched solves for each candidate and returns the fastest
    as ``{"blocks", "rows_per_tile", "weight_exponent", "persistent", "ms"}``."""
    key = batch_signature(batch, rtol)
    if key in _MEMO:
        return _MEMO[key]
    if cache_file and os.path.exists(cache_file):
        with open(cache_file) as f:
            disk = json.load(f)
        if key in disk:
            _MEMO[key] = disk[key]
            return disk[key]
    cus = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
    cands = list(candidates) if candidates is not None else default_candidates(cus)
    best = None
    x = torch.zeros_like(b)
    for c in cands:
        times = []
        try:
            for _ in range(repeats + 1):  # first run warms the shape up
                x.zero_()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                batch.batch_cg(b, x=x, rtol=rtol, maxit=maxit, blocks=c.blocks,
                               rows_per_tile=c.rows_per_tile, weight_exponent=c.weight_exponent,
                               persistent=c.persistent)
                torch.cuda.synchronize()
                times.append((time.perf_counter() - t0) * 1e3)
        except spx.SpxError as e:
            if e.code != spx.INVALID_ARG:  # a form this batch cannot take is skipped
                raise
            continue
        ms = min(times[1:])
        if verbose:
            print(f"[autotune] {asdict(c)} -> {ms:.3f} ms", flush=True)
        if best is None or ms < best["ms"]:
            best = dict(asdict(c), ms=ms)
    _MEMO[key] = best
    if cache_file:
        disk = {}
        if os.path.exists(cache_file):
            with open(cache_file) as f:
                disk = json.load(f)
        disk[key] = best
        os.makedirs(os.path.dirname(os.path.abspath(cache_file)), exist_ok=True)
        with open(cache_file, "w") as f:
            json.dump(disk, f, indent=1)
    return best


def tune_spmm(A: "spx.Matrix", X: torch.Tensor, candidates: Iterable[int] = (16, 32, 64),
              repeats: int = 5, verbose: bool = False) -> dict:
    """Tile height of the staged 16-column product (``OPT_SPMM_TILE_ROWS``):
    times ``repeats`` products of the actual matrix with X at each height
    (the first product at a height builds that height's index and is not
    timed), leaves the fastest set on A and returns ``{"rows", "ms",
    "all"}``.  Every height gives the same bits, so only time decides.
    Cached in memory per (device, matrix shape)."""
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    key = f"spmm|{props.name}|{A.n}|{A.nnz}|{tuple(candidates)}"
    if key in _MEMO:
        A.set_option(spx.OPT_SPMM_TILE_ROWS, _MEMO[key]["rows"])
        return _MEMO[key]
    Y = torch.empty_like(X)
    times = {}
    for rows in candidates:
        A.set_option(spx.OPT_SPMM_TILE_ROWS, rows)
        A.spmm(X, Y)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(repeats)]
        for s, e in ev:
            s.record()
            A.spmm(X, Y)
            e.record()
        torch.cuda.synchronize()
        times[rows] = min(s.elapsed_time(e) for s, e in ev)
        if verbose:
            print(f"[autotune] spmm tile rows {rows} -> {times[rows]:.4f} ms", flush=True)
    best = min(times, key=times.get)
    A.set_option(spx.OPT_SPMM_TILE_ROWS, best)
    _MEMO[key] = {"rows": best, "ms": times[best], "all": times}
    return _MEMO[key]
