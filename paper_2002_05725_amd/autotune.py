"""Autotuner for the apply_H launch shape.

Knobs (syk_set_apply_tuning): the tile of rows a workgroup owns (2^tile_bits
rows; 256 threads own up to 8 rows each, so tile_bits 8..11 chooses the rows
per thread 1..8 and the width of the LDS source tile), the order in which
tiles are handed to the 8 XCDs (contiguous ranges per XCD, or the hardware's
round robin) and, for blocks of an even number of columns, whether one
workgroup serves two columns of one realisation (tile_bits 10 and 11).  Each candidate is timed with the library's HIP-event timing of
apply_H on the handle's own tables for the requested block width and dtype,
the fastest is installed on the handle, and the choice is cached in a JSON file
keyed by (device architecture, N, dtype, block width), so a later run installs
it without timing.

All arithmetic runs in the library; this module only chooses among launch
shapes that produce the same product (up to the order of FP64 row sums).
"""
from __future__ import annotations

import json
import os

import torch

from . import api

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_2002_05725_amd", "apply_tuning.json")


def candidates(N: int, nvec: int = 1) -> list[tuple[int, int, int]]:
    """(tile_bits, xcd_remap, cols_per_group) triples valid for N Majoranas
    (M = N/2 qubits) and a block of nvec columns: tiles of 2^8 .. 2^11 rows
    (fewer when M is smaller), both tile orders, one column per workgroup, and
    for an even nvec also two columns per workgroup on tiles of 2^10 and 2^11
    rows."""
    M = N // 2
    tbs = [tb for tb in (8, 9, 10, 11) if tb <= M] or [M]
    out = [(tb, x, 1) for tb in tbs for x in (1, 0)]
    if nvec >= 2 and nvec % 2 == 0:
        out += [(tb, x, 2) for tb in tbs if tb >= 10 for x in (1, 0)]
    return out


def cache_key(arch: str, N: int, dtype: torch.dtype, nvec: int) -> str:
    name = {torch.complex128: "c128", torch.complex64: "c64"}[dtype]
    return f"{arch}|N={N}|{name}|nvec={nvec}"


def read_cache(path: str) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        d = json.load(f)
    return d if isinstance(d, dict) else {}


def write_cache(path: str, key: str, entry: dict) -> None:
    d = read_cache(path)
    d[key] = entry
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def pick(timings: list[dict]) -> dict:
    """The fastest candidate (ties: the first listed)."""
    if not timings:
        raise ValueError("no candidate was timed")
    return min(timings, key=lambda r: r["ms"])


def _arch() -> str:
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(p, "gcnArchName", p.name)


def time_shape(terms: api.Terms, x: torch.Tensor, y: torch.Tensor, tile_bits: int, xcd_remap: int,
               reps: int, cols_per_group: int = 1) -> float:
    """Average ms of one apply_H call on x (HIP events on the call's stream)
    with this launch shape; the first call (which builds the shape's tables) is
    not timed."""
    api.set_apply_tuning(terms, tile_bits, xcd_remap, cols_per_group)
    api.apply_H(terms, x, y)
    torch.cuda.synchronize()
    api.timing_reset()
    api.timing_enable(True)
    try:
        for _ in range(reps):
            api.apply_H(terms, x, y)
        torch.cuda.synchronize()
    finally:
        api.timing_enable(False)
    n, ms = api.timing_read()
    api.timing_reset()
    if n != reps:
        raise RuntimeError(f"apply_H timing recorded {n} calls, expected {reps}")
    return ms / n


def tune_apply(terms: api.Terms, dtype: torch.dtype = torch.complex128, nvec: int = 1, reps: int = 3,
               cache: str | None = DEFAULT_CACHE, shapes: list[tuple[int, int, int]] | None = None,
               use_cache: bool = True) -> dict:
    """Chooses and installs the apply_H launch shape for `terms`, `dtype` and a
    block of `nvec` columns (timed with every column in realisation 0, so
    that two-column shapes apply).  With use_cache and a cached entry for this
    key, installs that entry without timing.  Returns the chosen entry
    {"tile_bits", "xcd_remap", "cols_per_group", "ms", "timed": [...]}."""
    if dtype not in (torch.complex128, torch.complex64):
        raise ValueError("dtype must be complex128 or complex64")
    if nvec < 1 or reps < 1:
        raise ValueError("nvec and reps must be >= 1")
    key = cache_key(_arch(), terms.N, dtype, nvec)
    if cache and use_cache:
        hit = read_cache(cache).get(key)
        if hit is not None:
            api.set_apply_tuning(terms, hit["tile_bits"], hit["xcd_remap"], hit.get("cols_per_group", 1))
            return hit
    shape = (terms.dim,) if nvec == 1 else (nvec, terms.dim)
    g = torch.Generator(device="cuda").manual_seed(0)
    x = torch.randn(shape, dtype=dtype, device="cuda", generator=g)
    y = torch.empty_like(x)
    timed = []
    for tb, xr, nc in (shapes or candidates(terms.N, nvec)):
        timed.append({"tile_bits": tb, "xcd_remap": xr, "cols_per_group": nc,
                      "ms": time_shape(terms, x, y, tb, xr, reps, nc)})
    del x, y
    best = dict(pick(timed))
    best["timed"] = timed
    api.set_apply_tuning(terms, best["tile_bits"], best["xcd_remap"], best["cols_per_group"])
    if cache:
        write_cache(cache, key, best)
    return best
