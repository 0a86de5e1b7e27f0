"""Autotuner front end: run ptd_autotune and keep the results in a JSON cache.

The cache file is $PTD_AUTOTUNE_CACHE, else ~/.cache/ptd/tuning.json.  Each
entry is keyed by the GPU architecture, n, dtype and Hermitian flag and holds
the chosen setting of the dense single-launch schedule.  load() applies every
entry for the running architecture to the library's registry; it runs at
import unless PTD_AUTOTUNE=0.
"""
from __future__ import annotations

import ctypes
import json
import os

from . import _native, api


def cache_path() -> str:
    return os.environ.get("PTD_AUTOTUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "ptd",
                                                                  "tuning.json")


def _key(arch: str, n: int, dtype_code: int, hermitian: bool) -> str:
    return "%s/n%d/%s/%s" % (arch, n, "c128" if dtype_code == api.C128 else "c64", "herm" if hermitian else "gen")


def _arch() -> str:
    return _native.lib().ptd_build_arch().decode()


def autotune(n: int, dtype_code: int, hermitian: bool = False, reps: int = 5, save: bool = True) -> dict:
    """Tune one point on the current GPU; returns the chosen setting."""
    import torch

    L = _native.lib()
    cfg, la, tried, adm = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    ms = ctypes.c_float()
    st = L.ptd_autotune(n, dtype_code, api.HERMITIAN if hermitian else 0, reps,
                        api._stream_handle(torch.device("cuda", torch.cuda.current_device()), None),
                        ctypes.byref(cfg), ctypes.byref(la), ctypes.byref(ms), ctypes.byref(tried), ctypes.byref(adm))
    _native.check(st, "ptd_autotune")
    rec = {"cfg": cfg.value, "lookahead": la.value, "ms": ms.value, "candidates": tried.value,
           "admitted": adm.value}
    dms, bms, spr, kept = ctypes.c_float(), ctypes.c_float(), ctypes.c_float(), ctypes.c_int()
    if L.ptd_autotune_report(n, dtype_code, api.HERMITIAN if hermitian else 0, ctypes.byref(dms), ctypes.byref(bms),
                             ctypes.byref(spr), ctypes.byref(kept)) == 1:
        rec.update({"default_ms": dms.value, "spread_ms": spr.value, "kept": bool(kept.value)})
    if n >= 11:
        rec.update(describe(n, dtype_code, hermitian, cfg.value))
    if save:
        path = cache_path()
        data = {}
        if os.path.exists(path):
            try:
                data = json.load(open(path))
            except (OSError, ValueError):
                data = {}
        data[_key(_arch(), n, dtype_code, hermitian)] = rec
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    return rec


def describe(n: int, dtype_code: int, hermitian: bool = False, cfg: int = 0) -> dict:
    """The single-launch schedule's reading of a setting (n = 11..15; cfg 0
    is the default): workgroup threads, the low WHT stages per phase-1 item
    (the stage split) and the X-patterns per group (the tile width T)."""
    th, kap, t = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    st = _native.lib().ptd_describe_tuning(n, dtype_code, api.HERMITIAN if hermitian else 0, cfg, ctypes.byref(th),
                                           ctypes.byref(kap), ctypes.byref(t))
    _native.check(st, "ptd_describe_tuning")
    return {"threads": th.value, "phase1_bits": kap.value, "phase2_bits": n - kap.value,
            "group_patterns": t.value}


def load(path: str | None = None) -> int:
    """Apply cached settings for this architecture; returns how many."""
    path = path or cache_path()
    if not os.path.exists(path):
        return 0
    try:
        data = json.load(open(path))
    except (OSError, ValueError):
        return 0
    arch = _arch()
    L = _native.lib()
    applied = 0
    for k, rec in data.items():
        parts = k.split("/")
        if len(parts) != 4 or parts[0] != arch:
            continue
        n = int(parts[1][1:])
        code = api.C128 if parts[2] == "c128" else api.C64
        flags = api.HERMITIAN if parts[3] == "herm" else 0
        if L.ptd_set_tuning(n, code, flags, int(rec["cfg"]), int(rec["lookahead"])) == 0:
            applied += 1
    return applied
