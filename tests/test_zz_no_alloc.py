"""rept_count_noalloc (the count for callers that cannot allocate: its slot table lives in the
library's static device array) equals rept_count with a caller workspace, bit for bit, on calls
in a row where a later input is smaller than an earlier one (the array keeps the previous
call's contents), and refuses a slot table larger than the array."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


def test_noalloc_equals_count_on_calls_in_a_row(cuda):
    import torch
    from paper_1811_09136_amd import rept
    big, n_big = synth.scaled_chung_lu(400_000, 31)
    cases = [
        (big, n_big, rept.Params(10, 40, 5)),                  # four groups: 8 bytes per stored edge
        (synth.config1_stream(), 2000, rept.Params(7, 3, 9)),  # smaller input, one group
        (synth.er(300, 3000, 3, 4), 300, rept.Params(3, 7, 2, per_proc=True)),
        (synth.er(300, 3000, 3, 4), 300, rept.Params(10, 320, 8)),  # 32 groups: four launches
    ]
    for e, n, P in cases:
        _say(f"noalloc vs count: E={len(e)} n={n} m={P.m} c={P.c} per_proc={P.per_proc}")
        g = rept.Graph(rept.to_device_edges(e, cuda), n)
        ref = g.count(P)
        out = g.outputs(P)
        for _ in range(2):  # two calls on the same input too
            out[0].fill_(-3)
            out[1].fill_(-3)
            rept.rept_count_noalloc(g.handle, P, out[0].data_ptr(), out[1].data_ptr(),
                                    torch.cuda.current_stream().cuda_stream)
            torch.cuda.synchronize()
            assert torch.equal(out[0], ref[0]) and torch.equal(out[1], ref[1])
        assert int(ref[0].sum()) > 0
        g.close()


def test_noalloc_refuses_a_table_over_the_array(cuda):
    from paper_1811_09136_amd import rept
    e, n = synth.scaled_chung_lu(9_000_000, 33)
    g = rept.Graph(rept.to_device_edges(e, cuda), n)
    P = rept.Params(10, 40, 1)  # 2 bytes x 4 groups x 9e6 edges > 64 MiB
    assert g.workspace_bytes(P) > 64 << 20
    out = g.outputs(P)
    _say("noalloc: table over the array")
    with pytest.raises(rept.ReptError) as ei:
        rept.rept_count_noalloc(g.handle, P, out[0].data_ptr(), out[1].data_ptr(), None)
    assert ei.value.code == rept.REPT_ENOMEM
    P1 = rept.Params(10, 10, 1)  # one group: 18 MB fits
    ref = g.count(P1)
    out1 = g.outputs(P1)
    rept.rept_count_noalloc(g.handle, P1, out1[0].data_ptr(), out1[1].data_ptr(), None)
    import torch
    torch.cuda.synchronize()
    assert torch.equal(out1[0], ref[0]) and torch.equal(out1[1], ref[1])
    g.close()
