"""The field update alone (the sweep kernel's flush, through the probe
library's C entry point): after a flip sequence the FP64 table must equal the
fields recomputed from the final spins, h[k][j] = sum_{i != j} J*(|i-j|)
[s_i = k], to the rounding of the updates; bad words are refused on the host.
The VALU issue-rate probe beside it runs every instruction it times."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fb():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1308_5426_amd import flush_bench

    flush_bench.probe()
    return flush_bench


def _fields(J, s, q):
    """The table's definition, column by column: h[k][j] = sum_{i != j}
    J*(|i - j|) [s_i = k], with J*(0) = 0 and J* periodic."""
    L = len(s)
    h = np.zeros((q, L))
    idx = np.arange(L)
    for j in range(L):
        h[:, j] = np.bincount(s, weights=J[(idx - j) % L], minlength=q)
    return h


@pytest.mark.parametrize("L,q,n", [(256, 3, 3000), (1000, 4, 4097), (2, 2, 65), (1024, 2, 64), (3000, 3, 701)])
def test_replay_matches_recomputed_fields(fb, orc, L, q, n):
    J = np.asarray(orc.jstar(L, 0.4))
    words, s = workloads.flip_sequence(L, q, n, seed=L + q)
    h, ms = fb.replay(J, q, words, workgroups=3, reps=1)
    ref = _fields(J, s, q)
    np.testing.assert_allclose(h, ref, rtol=0, atol=1e-9 * max(1.0, float(np.abs(ref).max())))
    assert ms > 0.0


def test_replay_empty_sequence_keeps_table(fb, orc):
    J = np.asarray(orc.jstar(64, 0.6))
    h, _ = fb.replay(J, 3, np.zeros(0, np.uint32), workgroups=1, reps=1)
    ref = np.zeros((3, 64))
    ref[0, :] = J[1:].sum()
    np.testing.assert_array_equal(h, ref)


def test_replay_refuses_bad_words(fb, orc):
    J = np.asarray(orc.jstar(64, 0.6))
    with pytest.raises(RuntimeError):
        fb.replay(J, 3, np.array([64], np.uint32), workgroups=1, reps=1)  # site 64 of 64
    with pytest.raises(RuntimeError):
        fb.replay(J, 3, np.array([5 | (3 << 20)], np.uint32), workgroups=1, reps=1)  # state 3 of q = 3


@pytest.mark.parametrize("kind", ["fp64_fma", "fp32_fma"])
@pytest.mark.parametrize("threads", [256, 512])
def test_valu_issue_probe_runs_every_instruction(fb, kind, threads):
    """The issue-rate probe's checksum: 16 accumulators starting at 0..15, each
    updated iters times by x * 1 + 1, sum to 120 + 16 iters exactly."""
    ns, total = fb.valu_issue(kind, threads, iters=4096, blocks=8)
    assert total == 120 + 16 * 4096
    assert ns > 0.0


def test_valu_issue_probe_refuses_bad_arguments(fb):
    import ctypes

    ms, s = ctypes.c_double(), ctypes.c_double()
    lib = fb.probe()
    assert lib.ptmi_valu_issue_rate(2, 1, 256, 10, ctypes.byref(ms), ctypes.byref(s)) == -1  # no such kind
    assert lib.ptmi_valu_issue_rate(0, 1, 100, 10, ctypes.byref(ms), ctypes.byref(s)) == -1  # not whole waves
    assert lib.ptmi_valu_issue_rate(0, 1, 256, (1 << 20) + 1, ctypes.byref(ms), ctypes.byref(s)) == -1
