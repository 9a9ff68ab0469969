"""The library's per-stream state (workspace, plan cache, pinned staging):
every entry point gives the same bits on a side stream as on the default
stream, and work queued on two streams at once does not mix."""
import numpy as np
import pytest

import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ph():
    import paper_1606_05836_amd as ph

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return ph


def cuda(a):
    return torch.from_numpy(np.array(a, copy=True)).to("cuda")


def run_all(ph, a, b, u, ins, pats):
    n = a.shape[0]
    perms, unis = ph.sample_inputs(8, len(ins), 3)
    return (ph.perm(a), ph.perm_batched(b), ph.perm_grad(b[:4])[1], ph.boson_probs(u, ins, pats),
            ph.boson_probs_grad(u, ins, pats)[1], ph.perm_partial(a, 0, ph.gray_terms(n) // 2),
            ph.perm_row_minors(b[:4, :15, :]), ph.boson_sample(u, ins, perms=perms, uniforms=unis))


def test_side_stream_gives_the_same_bits(ph):
    a = cuda(I.haar1600_block(24))
    b = cuda(I.grad_batch_20(32, 16))
    u_np, ins, pats = I.boson_workload(m=200, n=16, patterns=6)
    u = cuda(u_np)
    ref = [x.cpu() for x in run_all(ph, a, b, u, ins, pats)]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        got = run_all(ph, a, b, u, ins, pats)
    side.synchronize()
    for r, g in zip(ref, got):
        assert torch.equal(r, g.cpu())


def test_two_streams_in_flight(ph):
    # different work on two streams at once, each checked against its own
    # default-stream result
    m1 = cuda(I.grad_batch_20(64, 18))
    m2 = cuda(I.haar1600_block(26))
    r1 = ph.perm_batched(m1).cpu()
    r2 = ph.perm(m2).cpu()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    s1.wait_stream(torch.cuda.current_stream())
    s2.wait_stream(torch.cuda.current_stream())
    outs = []
    for _ in range(3):
        with torch.cuda.stream(s1):
            o1 = ph.perm_batched(m1)
        with torch.cuda.stream(s2):
            o2 = ph.perm(m2)
        outs.append((o1, o2))
    s1.synchronize()
    s2.synchronize()
    for o1, o2 in outs:
        assert torch.equal(o1.cpu(), r1)
        assert torch.equal(o2.cpu(), r2)


def test_one_plan_on_two_streams_back_to_back(ph):
    # a plan's counters and partials are its own: a replay on a second stream
    # must wait for the replay still running on the first
    ns, mats = I.mixed_batch_16_26(batch=512)
    flat = torch.cat([cuda(m).reshape(-1) for m in mats])
    plan = ph.Plan(ns)
    ref = plan(flat).cpu()
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    s1.wait_stream(torch.cuda.current_stream())
    s2.wait_stream(torch.cuda.current_stream())
    outs = []
    for _ in range(4):
        for s in (s1, s2):
            with torch.cuda.stream(s):
                outs.append(plan(flat))
    s1.synchronize()
    s2.synchronize()
    for o in outs:
        assert torch.equal(o.cpu(), ref)
    plan.close()


def test_binding_rejects_mismatched_device_buffers(ph):
    # sizes the C ABI cannot see are checked by the binding before the call
    a = cuda(I.haar1600_block(12))
    with pytest.raises(ValueError, match="1 elements"):
        ph.perm(a, out=torch.empty(2, dtype=torch.complex128, device="cuda"))
    with pytest.raises(TypeError, match="complex128"):
        ph.perm(a, out=torch.empty((), dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError, match="1 elements"):
        ph.perm_ryser_paired(a, out=torch.empty(3, dtype=torch.complex128, device="cuda"))
    with pytest.raises(ValueError, match="n x n"):
        ph.perm_batched([a, a[:, :11]])
    plan = ph.Plan([12, 12])
    with pytest.raises(ValueError, match="reads 288"):
        plan(a.reshape(-1))  # one matrix where the plan reads two
    with pytest.raises(ValueError, match="2 elements"):
        plan(torch.cat([a.reshape(-1), a.reshape(-1)]), out=torch.empty(1, dtype=torch.complex128, device="cuda"))
    good = plan(torch.cat([a.reshape(-1), a.reshape(-1)]))
    assert torch.equal(good[0], good[1])
    plan.close()
    with pytest.raises(ValueError, match="4 elements"):
        ph.perm_partial(a, 0, 0, out=torch.empty(3, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError, match="1 elements"):
        ph.perm_combine(torch.zeros(2, 4, dtype=torch.float64, device="cuda"), 12,
                        out=torch.empty(4, dtype=torch.complex128, device="cuda"))
