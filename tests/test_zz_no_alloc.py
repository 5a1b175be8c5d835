"""treepm_timestep_noalloc (the allocation-free variant of treepm_timestep, its reduction word
in a static device array of the library) against treepm_timestep and the FP64 oracle: the
shared step of eq. (7) bit for bit, on two calls in a row on one GPU -- the second with a
smaller input whose step is longer, so a reduction word left over from the first call would
show -- and with a context that never allocated the time step's own buffer."""
import sys

import numpy as np
import pytest

import boxgen
from oracle import integrate as it

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

ERR_ARG = -1  # TREEPM_ERR_ARG of include/treepm.h


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0910_0121_amd as t
    t.lib()
    return t


def _ctx(tp):
    mesh = 1.0 / 32
    return tp.treepm_create(tp.make_params(1.0, mesh, 3 * mesh, 1e-4, 0.5, 10, 64,
                                           tp.TREEPM_FP64), 0)


def _arrays(n, seed, amp, dtype):
    rng = boxgen.SplitMix64(seed)
    v = rng.uniform(3 * n).reshape(n, 3) - 0.5
    a = ((rng.uniform(3 * n).reshape(n, 3) - 0.5) * amp).astype(dtype)
    a[3] = 0.0
    v[5] = 0.0
    return v, a


def test_noalloc_timestep_matches_the_allocating_call(tp):
    ctx_ref, ctx_na = _ctx(tp), _ctx(tp)
    try:
        cases = [(300007, 21, 1e6, np.float64), (1001, 22, 1e-2, np.float32)]
        dts = []
        for n, seed, amp, dt_ in cases:
            _say(f"timestep_noalloc n={n} acc={np.dtype(dt_).name}")
            v, a = _arrays(n, seed, amp, dt_)
            vd = [torch.from_numpy(np.ascontiguousarray(v[:, c])).cuda() for c in range(3)]
            ad = [torch.from_numpy(np.ascontiguousarray(a[:, c])).cuda() for c in range(3)]
            got = tp.treepm_timestep_noalloc(ctx_na, *vd, *ad, 1e-4, 0.3)
            ref = tp.treepm_timestep(ctx_ref, *vd, *ad, 1e-4, 0.3)
            orc = it.timestep(v, a.astype(np.float64), 1e-4, 0.3)
            assert got == ref == orc, (got, ref, orc)
            dts.append(got)
        assert dts[1] > dts[0]  # the second call's step is the longer one
        # argument errors are reported before anything runs
        import ctypes as C
        v, a = _arrays(10, 23, 1.0, np.float64)
        vh = [torch.from_numpy(np.ascontiguousarray(v[:, c])) for c in range(3)]
        ah = [torch.from_numpy(np.ascontiguousarray(a[:, c])) for c in range(3)]
        out = C.c_double(-1.0)
        rc = tp.lib().treepm_timestep_noalloc(ctx_na, 10, *[t.data_ptr() for t in vh + ah],
                                              tp.TREEPM_FP64, 1e-4, 0.3, None, C.byref(out))
        assert rc == ERR_ARG and out.value == -1.0  # host arrays are refused
        vd = [t.cuda() for t in vh]
        ad = [t.cuda() for t in ah]
        with pytest.raises(tp.TreePMError) as e:
            tp.treepm_timestep_noalloc(ctx_na, *vd, *ad, 0.0, 0.3)
        assert e.value.code == ERR_ARG
        # and the variant still works after the rejected calls
        assert tp.treepm_timestep_noalloc(ctx_na, *vd, *ad, 1e-4, 0.3) == \
            it.timestep(v, a, 1e-4, 0.3)
    finally:
        tp.treepm_destroy(ctx_ref)
        tp.treepm_destroy(ctx_na)
