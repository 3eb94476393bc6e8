"""Host-side checks of the batched form: the mixed-batch generator and the
C-ABI layout of the launch options (no GPU)."""
import ctypes
import os

import numpy as np

import batch_util as B
from oracle import oracle as O
from paper_2601_01048_amd import ckc
from paper_2601_01048_amd.gen import workloads as W


def test_launch_opts_layout():
    assert ctypes.sizeof(ckc.LaunchOpts) == 32
    assert ctypes.sizeof(ckc.TuneEntry) == 40


def test_exports():
    L = ckc.lib()
    for f in ("ckc_job_elapsed", "ckc_autotune"):
        assert hasattr(L, f)


def test_config4_shapes():
    mb = W.config4(n_kernels=400)
    T = mb.meta["T"]
    assert T.min() >= 1 and T.max() <= 65536
    assert set(np.unique(mb.meta["family"])) == {0, 1, 2}
    for k in mb.kernels:
        t = k.meta["T"]
        L = k.launch[0].astype(np.int64)
        threads = int(np.prod(L))
        if k.meta["family"] == "F1":
            assert L[3] == min(256, t) and L[0] == -(-t // L[3])
            assert -(-9 * t // 10) <= k.meta["n"] <= -(-11 * t // 10)
        elif k.meta["family"] == "F2":
            side = int(np.ceil(np.sqrt(t)))
            assert L[3] == L[4] == min(16, side) and threads >= t
        else:
            assert k.meta["nnz"] == min(16 * t, t * t)
            assert threads >= t
        w64 = k.name.endswith("i64")
        if w64:
            assert k.scalars[0, -1] == W.I64_BASE


def test_group_matches_single_oracle_runs():
    """The grouped oracle call gives each kernel the result of its own call."""
    mb = W.config4(seed=11, n_kernels=24, t_max=300)
    grouped = B.oracle_mixed(mb)
    for i, k in enumerate(mb.kernels):
        single = O.check(k)
        B.same(grouped[i], dict(records=single["records"][0], maps=single["maps"][0],
                                status=single["status"][0]), f"kernel {i}")


def test_config5_stream_shape():
    ss = W.config5(duration_s=2.0)
    gaps = np.diff(ss.arrivals)
    assert abs(ss.n_jobs / 2.0 - 2000) < 150           # Poisson count, 2000/s over 2 s
    assert abs(gaps.mean() - 1 / 2000) < 5e-5
    A = ss.meta["A"]
    assert A.min() >= 1e3 and A.max() <= 1e7
    assert abs(np.log(A).mean() - 0.5 * (np.log(1e3) + np.log(1e7))) < 0.15
    for k in ss.jobs:
        if k.meta["family"] == "F3":
            nr = k.meta["T"]
            assert nr == 1 << k.meta["log2_rows"] and 4 <= k.meta["log2_rows"] <= 18
            assert abs(k.meta["x"] - nr) <= 64
            refs = k.tables[0]["data"]
            assert refs[0] >= 1 and refs[1] == refs[0] + 1


def test_server_struct_layouts():
    assert ctypes.sizeof(ckc.ServerConfig) == 48
    assert ctypes.sizeof(ckc.JobStats) == 40
    assert ctypes.sizeof(ckc.ServerStats) == 48


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU: --gpus above 1 ends with a message and
    a nonzero status, before touching a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
