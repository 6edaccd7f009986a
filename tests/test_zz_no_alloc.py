"""ffs_decode_noalloc (the decode on the library's own per-GPU scratch buffer)
against ffs_decode with a caller workspace, through the C ABI, bit for bit.

Two calls in a row share the buffer (the second on a smaller input), with the
on-chip profile cut short so the overflow tier, whose counters live in the
buffer's header, runs too; an input whose workspace exceeds the buffer is
rejected before anything is launched.
"""
import numpy as np
import pytest

import oracle
from paper_1903_10741_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


def _both(ffsga, torch, inst, pop, lds_slots):
    d = ffsga.DeviceInstance.from_host(inst)
    prio = torch.from_numpy(pop).cuda()
    ref = ffsga.ffs_decode(d, prio, lds_slots=lds_slots, want_schedule=True, want_work=True)
    got = ffsga.ffs_decode_noalloc(d, prio, lds_slots=lds_slots, want_schedule=True,
                                   want_work=True)
    torch.cuda.synchronize()
    for k in ("obj", "work", "start", "mach"):
        assert torch.equal(got[k], ref[k]), k
    return got


def test_noalloc_matches_workspace_decode_twice():
    import torch
    from paper_1903_10741_amd import ffsga
    assert torch.cuda.is_available()
    big = W.config2(0).initial
    small = W.config1(0).initial
    _say("noalloc: paper-50x5x3 pop 512, 64 on-chip slots (overflow tier)")
    pop_big = W.random_population(21, 512, big.n_active)
    got = _both(ffsga, torch, big, pop_big, 64)
    obj = got["obj"].cpu().numpy()
    for i in range(0, 512, 64):   # and against the oracle on a sample
        assert obj[i] == oracle.decode(big, pop_big[i]), i
    _say("noalloc: tiny-10x2x2 pop 64, default slots (second call, smaller input)")
    pop_small = W.random_population(22, 64, small.n_active)
    got = _both(ffsga, torch, small, pop_small, 0)
    obj = got["obj"].cpu().numpy()
    assert (obj == oracle.decode_pop(small, pop_small)).all()
    _say("noalloc: paper-50x5x3 pop 96, default slots (third call)")
    _both(ffsga, torch, big, W.random_population(23, 96, big.n_active), 0)


def test_noalloc_rejects_a_workspace_beyond_the_buffer():
    import torch
    from paper_1903_10741_amd import ffsga
    inst = W.config1(0).initial
    d = ffsga.DeviceInstance.from_host(inst)
    # 64 on-chip slots below the horizon: the overflow list takes 4 bytes per chromosome
    pop = (ffsga.FFS_DECODE_SCRATCH_BYTES // 4) + 64
    assert d.horizon > 64
    need = ffsga._lib.ffs_decode_workspace_size(ctypes_ref(d), pop, 64)
    assert need > ffsga.FFS_DECODE_SCRATCH_BYTES
    _say("noalloc: reject pop", pop, "needing", need, "bytes")
    prio = torch.from_numpy(np.tile(np.arange(1, inst.n_active + 1, dtype=np.int32),
                                    (pop, 1))).cuda()
    with pytest.raises(ffsga.FfsError) as e:
        ffsga.ffs_decode_noalloc(d, prio, lds_slots=64)
    assert e.value.code == ffsga.FFS_E_WORKSPACE


def ctypes_ref(d):
    import ctypes
    return ctypes.byref(d.s)
