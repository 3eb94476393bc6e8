"""Cache of autotuned launch options.

ckc_autotune times launch-option candidates on a batch and returns the
fastest.  Tuning costs tens of jobs, so the choice is kept as JSON keyed by
the GPU architecture (e.g. ``gfx950``) and a coarse signature of the batch:
the set of programs, the number of descriptors and the total thread count,
each rounded to a power of two.  Two batches drawn from one recipe with
different seeds share a signature, which is what lets a batch be tuned on
one seed and measured on another.  Host-side bookkeeping only.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

from . import ckc


def cache_path() -> str:
    p = os.environ.get("CKC_TUNE_CACHE")
    return p or os.path.join(os.path.expanduser("~"), ".cache", "ckc", "autotune.json")


def gfx_arch(device: int = 0) -> str:
    import torch
    return torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]


def _pow2(n: int) -> int:
    return 0 if n <= 0 else int(n).bit_length()


def signature(irs, launches) -> str:
    """irs: program bytes per descriptor; launches: [n, 6] launch rows of
    every input of the batch."""
    progs = sorted({hashlib.sha256(ir).hexdigest()[:12] for ir in irs})
    L = np.asarray(launches, np.uint64).reshape(-1, 6)
    threads = int((L[:, 0] * L[:, 1] * L[:, 2] * L[:, 3] * L[:, 4] * L[:, 5]).sum())
    key = dict(progs=progs, descs_log2=_pow2(len(irs)), inputs_log2=_pow2(len(L)), threads_log2=_pow2(threads))
    return hashlib.sha256(json.dumps(key, sort_keys=True).encode()).hexdigest()[:16]


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def lookup(arch: str, sig: str, path: str | None = None):
    """The cached entry for (arch, sig) or None."""
    return _load(path or cache_path()).get(arch, {}).get(sig)


def store(arch: str, sig: str, opts: ckc.LaunchOpts, ms: float, note: str, path: str | None = None):
    path = path or cache_path()
    data = _load(path)
    data.setdefault(arch, {})[sig] = dict(schedule=int(opts.schedule), chunk=int(opts.chunk),
                                          wg_per_cu=int(opts.wg_per_cu), ms=float(ms), note=note)
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def opts_of(entry: dict) -> ckc.LaunchOpts:
    return ckc.launch_opts(entry["schedule"], entry["chunk"], entry["wg_per_cu"])


def tuned(ctx: ckc.Context, tune_descs, arch: str, sig: str, note: str, reps: int = 1, path: str | None = None):
    """Launch options for batches of signature ``sig``: from the cache, else
    tuned on ``tune_descs`` (a prepared batch other than the one to be
    measured) and stored.  Returns (opts, dict describing where they came
    from, tuning log or None)."""
    hit = lookup(arch, sig, path)
    if hit is not None:
        return opts_of(hit), dict(source="cache", **hit), None
    best, log = ctx.autotune(tune_descs, reps=reps)
    ms = min(m for _, m in log)
    store(arch, sig, best, ms, note, path)
    return best, dict(source="tuned", schedule=int(best.schedule), chunk=int(best.chunk),
                      wg_per_cu=int(best.wg_per_cu), ms=ms, note=note), log
