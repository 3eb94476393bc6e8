"""The entry point that allocates nothing (ckc_check_batch_noalloc), for
callers that cannot allocate device memory, against ckc_check_batch +
ckc_read_results on the same descriptors: records, maps and status must be
byte-identical.  Each case makes two calls in a row, the second with fewer
inputs, so the second runs over the first call's leftovers in the shared
scratch; output buffers start filled with garbage."""
import numpy as np
import pytest

from paper_2601_01048_amd import ckc
from paper_2601_01048_amd.gen import workloads as W

pytestmark = pytest.mark.gpu

GARBAGE = 0xCD


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = ckc.Context(0)
    yield c
    c.close()


def noalloc(ctx, descs, n_inputs, n_rec, dense, opts=None):
    import torch
    recs = torch.full((max(1, n_rec) * 32,), GARBAGE, dtype=torch.uint8, device="cuda")
    st = torch.full((n_inputs * 40,), GARBAGE, dtype=torch.uint8, device="cuda")
    maps = torch.full((n_inputs * 65536,), GARBAGE, dtype=torch.uint8, device="cuda") if dense else None
    torch.cuda.synchronize()  # the fills run on torch's stream, the check on the library's
    ctx.check_noalloc(descs, recs.data_ptr(), maps.data_ptr() if dense else None, st.data_ptr(), opts)
    torch.cuda.synchronize()
    r = np.frombuffer(recs.cpu().numpy().tobytes(), ckc.RECORD_DTYPE)[:n_rec]
    s = np.frombuffer(st.cpu().numpy().tobytes(), ckc.STATUS_DTYPE)
    m = maps.cpu().numpy().reshape(n_inputs, 65536) if dense else None
    return r, m, s


def reference(ctx, descs, dense, opts=None):
    job = ctx.check(descs, opts=opts)
    return ctx.read(job, maps=dense)


def same(got, ref, what):
    (gr, gm, gs), (rr, rm, rs) = got, ref
    assert gr.tobytes() == rr.tobytes(), f"{what}: records differ"
    assert gs.tobytes() == rs.tobytes(), f"{what}: status differs"
    if rm is not None:
        assert np.array_equal(gm, rm), f"{what}: maps differ"


def n_records(dw, n_inputs):
    return n_inputs * dw.info["n_accesses"]


CASES = [("config2", ckc.FULL, False), ("config2", ckc.REP_BOUNDARY, False), ("config2", ckc.REP_CORNERS, False),
         ("config2", ckc.FULL, True), ("config1", ckc.FULL, False), ("config3", ckc.FULL, False)]


@pytest.mark.parametrize("name,mode,generic", CASES)
def test_noalloc_equals_check_batch_twice(ctx, name, mode, generic):
    wl = W.mini(name)
    n = wl.n_inputs
    print(f"[case] noalloc {name} mode={mode} generic={generic} inputs={n} then {n // 2}", flush=True)
    dw = ckc.DeviceWorkload(ctx, wl)
    opts = ckc.launch_opts(force_generic=generic)
    try:
        for k, idx in enumerate((slice(None), slice(0, n // 2))):
            desc = [dw.desc(mode=mode, dense=True, idx=idx)]
            m = len(range(n)[idx])
            ref = reference(ctx, desc, True, opts)
            got = noalloc(ctx, desc, m, n_records(dw, m), True, opts)
            same(got, ref, f"{name} call {k}")
            assert int(got[2]["accesses_checked"].sum()) > 0
    finally:
        dw.close()


def test_noalloc_mixed_descriptors_without_maps(ctx):
    """Many descriptors of different programs (both widths, the three
    families) in one call, then a smaller call; no dense maps."""
    mb = W.config4(seed=1004, n_kernels=90, t_max=4096)
    print(f"[case] noalloc mixed batch of {mb.n_kernels} kernels then 30", flush=True)
    db = ckc.DeviceBatch(ctx, mb)
    try:
        for k, idx in enumerate((None, list(range(30, 60)))):
            descs = db.descs(idx, dense=False)
            ks = range(mb.n_kernels) if idx is None else idx
            nrec = sum(db.n_accesses(i) for i in ks)
            ref = reference(ctx, descs, False)
            got = noalloc(ctx, descs, len(descs), nrec, False)
            same(got, ref, f"mixed call {k}")
    finally:
        db.close()


def test_noalloc_full_size_csr_input(ctx):
    """One input of the CSR workload at its full size (2^20 rows, power-law
    rows): the largest expanded-loop state that fits in the scratch."""
    wl = W.config3(n_inputs=1)
    print("[case] noalloc CSR 2^20 rows, one input", flush=True)
    dw = ckc.DeviceWorkload(ctx, wl)
    try:
        desc = [dw.desc(dense=True)]
        ref = reference(ctx, desc, True)
        got = noalloc(ctx, desc, 1, n_records(dw, 1), True)
        same(got, ref, "csr full size")
        col = wl.data[1]
        bad = int(((col < 0) | (col >= wl.meta["ncols"])).sum())
        assert int(got[0]["count"][1:].sum()) >= bad  # the x[col] access flags every bad column
    finally:
        dw.close()


def test_noalloc_rejections(ctx):
    """Sizes beyond the limits and unsupported options are refused before
    anything is queued."""
    import torch
    print("[case] noalloc rejections", flush=True)
    wl = W.mini("config2")
    dw = ckc.DeviceWorkload(ctx, wl)
    buf = torch.zeros(1 << 20, dtype=torch.uint8, device="cuda")
    p = buf.data_ptr()
    try:
        too_many = dw.desc(dense=False, idx=np.zeros(4097, np.int64))
        with pytest.raises(ckc.CkcError) as e:
            ctx.check_noalloc([too_many], p, None, p)
        assert e.value.code == -1 and "4096" in str(e.value)
        with pytest.raises(ckc.CkcError) as e:  # dense maps asked for, no buffer
            ctx.check_noalloc([dw.desc(dense=True)], p, None, p)
        assert e.value.code == -1
        with pytest.raises(ckc.CkcError) as e:  # a map buffer without dense maps
            ctx.check_noalloc([dw.desc(dense=False)], p, p, p)
        assert e.value.code == -1
        with pytest.raises(ckc.CkcError) as e:
            ctx.check_noalloc([dw.desc(mode=ckc.REP_PREX, dense=False)], p, None, p)
        assert e.value.code == -1
        with pytest.raises(ckc.CkcError) as e:
            ctx.check_noalloc([dw.desc(dense=False)], p, None, p, ckc.launch_opts(use_graph=True))
        assert e.value.code == -1
        with pytest.raises(ckc.CkcError) as e:
            ctx.check_noalloc([dw.desc(dense=False)], 0, None, p)
        assert e.value.code == -1
    finally:
        dw.close()
    # expanded-loop state of four full-size CSR inputs exceeds the scratch
    big = W.config3(n_inputs=4)
    dw = ckc.DeviceWorkload(ctx, big)
    try:
        with pytest.raises(ckc.CkcError) as e:
            ctx.check_noalloc([dw.desc(dense=False)], p, None, p)
        assert e.value.code == -4 and "scratch" in str(e.value)
    finally:
        dw.close()
    # the context still works afterwards
    wl = W.mini("config1")
    dw = ckc.DeviceWorkload(ctx, wl)
    try:
        desc = [dw.desc(dense=True)]
        same(noalloc(ctx, desc, wl.n_inputs, n_records(dw, wl.n_inputs), True), reference(ctx, desc, True),
             "after rejections")
    finally:
        dw.close()
