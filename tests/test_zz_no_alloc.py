"""The allocation-free QR entry point (dcgs2_qr_noalloc) against dcgs2_qr, through the
C ABI: the same kernels on buffers in the library's fixed scratch array, so the
results must be identical, bit for bit, to dcgs2_qr's on the same input.  Two calls
in a row, the second with a smaller input, show that the scratch left by the first
call does not leak into the second."""
import numpy as np
import pytest

from paper_2104_01253_amd import binding, synth
from tests._gpu import dev_matrix, host, say, torch_cuda

pytestmark = pytest.mark.gpu


def _both(ctx, B, one_pass):
    Bd = dev_matrix(B)
    Q1 = binding.colmajor_empty(*B.shape)
    Q2 = binding.colmajor_empty(*B.shape)
    ctx.set_qr_schedule(one_pass)
    try:
        R1, rc1, st1 = ctx.qr(Bd, Q1)
        R2, rc2, st2 = ctx.qr_noalloc(Bd, Q2)
    finally:
        ctx.set_qr_schedule(True)
    return (host(Q1), R1, rc1, st1), (host(Q2), R2, rc2, st2)


@pytest.mark.parametrize("one_pass", [True, False])
def test_qr_noalloc_matches_qr_twice(one_pass):
    torch_cuda()
    with binding.Context(0) as ctx:
        for m, n, ce in [(2_000_000, 100, 8), (30011, 17, 4)]:
            say(f"noalloc qr m={m} n={n} one_pass={one_pass}")
            B = synth.tall_skinny(m, n, ce, seed_g=900 + n, seed_v=3)
            (Q1, R1, rc1, st1), (Q2, R2, rc2, st2) = _both(ctx, B, one_pass)
            assert rc1 == rc2 == binding.OK
            assert st1["reductions"] == st2["reductions"] == n + 1
            assert np.array_equal(R1, R2) and np.array_equal(Q1, Q2)


def test_qr_noalloc_fresh_context_limits_and_breakdown():
    """A context whose first call is the allocation-free one; the largest accepted
    size and the breakdown prefix."""
    torch_cuda()
    with binding.Context(0) as ctx:
        B = synth.tall_skinny(2 ** 21, 128, 4, seed_g=31, seed_v=32)
        Bd = dev_matrix(B)
        Q = binding.colmajor_empty(*B.shape)
        R2, rc2, _ = ctx.qr_noalloc(Bd, Q)
        Q2 = host(Q)
    with binding.Context(0) as ctx:
        R1, rc1, _ = ctx.qr(Bd, Q)
        assert rc1 == rc2 == binding.OK
        assert np.array_equal(R1, R2) and np.array_equal(host(Q), Q2)
        Bb = synth.tall_skinny(5000, 8, 2)
        Bb[:, 3] = Bb[:, 0] - 2.0 * Bb[:, 2]
        (Q1, R1, rc1, st1), (Qn, Rn, rcn, stn) = _both(ctx, Bb, True)
        assert rc1 == rcn == binding.BREAKDOWN
        assert st1["breakdown_step"] == stn["breakdown_step"] == 3
        assert np.array_equal(R1[:3, :4], Rn[:3, :4])
        assert np.array_equal(Q1[:, :3], Qn[:, :3])
        with pytest.raises(ValueError):
            ctx.qr_noalloc(Bd[:, :10], Q[:, :9])
