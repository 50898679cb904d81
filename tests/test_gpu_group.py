"""Grouped solves: one launch per kernel serves several same-shape controllers (slots of
one group).  Each slot's result is bitwise the same alone (its own solve), in any batch of
the group, and on a plain handle with the same inputs; against the FP64 oracle it meets the
BF16 bar like any BF16 solve.

The shapes cover the serving mix's kernel families: 16-channel tanh CNN with the
one-workgroup Cholesky (p <= 90) and the row update; 32-channel GELU CNN with the BF16
row-pair kernel; p > 90 with the blocked Cholesky chain and the strip update; 64-channel
GELU CNN with the last layer folded into the last hidden layer; ragged field sizes."""
import dataclasses

import numpy as np
import pytest

from oracle import enks
from paper_2410_09663_amd import oic
from paper_2410_09663_amd import workloads as wl
from parity_util import assert_parity

pytestmark = pytest.mark.gpu

FAMILIES = {
    # p = 36: one-workgroup Cholesky, row update; 16 -> 16 BF16 hidden layer; ragged tiles
    "c16_ragged": wl.small_preset(n=30, m=36, l=6, channels=(2, 16, 16, 1), N=24, H=3),
    # p = 80, 32 channels: row-pair BF16 kernel
    "c32": wl.small_preset(n=64, m=64, l=16, channels=(2, 32, 32, 32, 1), activation=wl.ACT_GELU, N=16, H=2),
    # p = 160: blocked Cholesky chain, strip update with the split gain
    "c32_p160": wl.small_preset(n=128, m=64, l=32, channels=(2, 32, 32, 32, 1), activation=wl.ACT_GELU,
                                N=8, H=2),
    # 64 channels, last layer folded into the last hidden layer (tap sum)
    "c64_fold": wl.small_preset(n=48, m=64, l=12, channels=(2, 64, 64, 64, 64, 1), activation=wl.ACT_GELU,
                                N=8, H=2),
}


def _problems(p, count):
    """count controllers of one shape with their own B, weights and X0."""
    return [wl.make_problem(dataclasses.replace(p, name=f"{p.name}{i}", seed_B=30 + 3 * i, seed_W=31 + 3 * i,
                                                seed_X0=32 + 3 * i)) for i in range(count)]


def _biases(prob, seed):
    rng = np.random.default_rng(seed)
    return [(0.05 * rng.standard_normal(co)).astype(np.float32) for co in prob.preset.channels[1:]]


def _request(prob, k):
    p = prob.preset
    X0 = (prob.X0 * (1.0 + 0.1 * k)).astype(np.float32)
    U_prev = np.full((p.l, p.m), 0.01 * k, np.float32)
    return dict(X0=X0, reference=wl.reference_window(p, k), Q=prob.Q, R=prob.R, N=p.N, H=p.H,
                seed=1000 + 17 * k, U_prev=U_prev, want_X=True)


@pytest.mark.parametrize("family", list(FAMILIES))
def test_group_slots_match_their_own_solves_bitwise(family):
    p = FAMILIES[family]
    G = 3
    probs = _problems(p, G)
    bias = [None, _biases(probs[1], 5), None]  # slot 1 with biases, the others without
    print(f"group {family}: n={p.n} m={p.m} l={p.l} channels={p.channels} N={p.N} H={p.H}", flush=True)
    with oic.Group(p.n, p.m, p.l, p.channels, p.activation, p.N, p.H, G) as grp:
        for i, pr in enumerate(probs):
            grp.slots[i].set_weights(pr.B, pr.weights, bias[i])
        reqs = [_request(pr, i) for i, pr in enumerate(probs)]
        alone = [grp.slots[i].solve_ex(**reqs[i]) for i in range(G)]
        # the same solve on a plain handle (own allocations, no bias instead of a zero one)
        for i, pr in enumerate(probs):
            with oic.Controller(p.n, p.m, p.l, p.channels, p.activation, p.N, p.H,
                                precision=oic.OIC_PREC_BF16) as c:
                c.set_weights(pr.B, pr.weights, bias[i])
                U, X = c.solve_ex(**reqs[i])
            assert np.array_equal(U, alone[i][0]) and np.array_equal(X, alone[i][1]), ("plain", i)
        # every slot in one batch, then subsets in other orders; the captured grouped solve
        # is replayed with eager work (solves of single slots) between the replays
        for batch in ([0, 1, 2], [2, 0], [1], [0, 1, 2], [1, 2]):
            outs = grp.solve([(i, reqs[i]) for i in batch])
            for i, (U, X) in zip(batch, outs):
                assert np.array_equal(U, alone[i][0]), (batch, i)
                assert np.array_equal(X, alone[i][1]), (batch, i)
            assert grp.rc_codes == [0] * len(batch)
            one = grp.slots[2].solve_ex(**reqs[2])
            assert np.array_equal(one[0], alone[2][0])


def test_group_with_explicit_noise_meets_the_bf16_bar_against_the_oracle():
    p = FAMILIES["c16_ragged"]
    probs = _problems(p, 2)
    noise = [wl.host_noise(p.n, p.m, p.l, p.N, p.H, seed=40 + i) for i in range(2)]
    with oic.Group(p.n, p.m, p.l, p.channels, p.activation, p.N, p.H, 2) as grp:
        reqs = []
        for i, pr in enumerate(probs):
            grp.slots[i].set_weights(pr.B, pr.weights)
            reqs.append(dict(X0=pr.X0, reference=wl.reference_window(p, 0), Q=pr.Q, R=pr.R, N=p.N, H=p.H,
                             noise=noise[i], U_prev=np.zeros((p.l, p.m), np.float32), want_X=True))
        outs = grp.solve([(0, reqs[0]), (1, reqs[1])])
    for i, pr in enumerate(probs):
        z = noise[i]
        ref = enks.solve(pr.B, pr.weights, p.activation, pr.X0, wl.reference_window(p, 0), pr.Q, pr.Q, pr.R,
                         p.N, p.H, z.Z_init, z.Z_W, z.Z_VX, z.Z_VU)
        eu, eu_max = assert_parity(outs[i][0], ref.U_mean, 2e-2, "U")
        ex, ex_max = assert_parity(outs[i][1], ref.X_mean, 2e-2, "X")
        print(f"grouped slot {i} vs oracle: relerr U {eu:.2e} (max {eu_max:.2e}) X {ex:.2e} (max {ex_max:.2e})",
              flush=True)


def test_a_request_that_differs_fails_alone():
    p = FAMILIES["c16_ragged"]
    probs = _problems(p, 3)
    with oic.Group(p.n, p.m, p.l, p.channels, p.activation, p.N, p.H, 3) as grp:
        for i, pr in enumerate(probs):
            grp.slots[i].set_weights(pr.B, pr.weights)
        reqs = [_request(pr, i) for i, pr in enumerate(probs)]
        alone = [grp.slots[i].solve_ex(**reqs[i]) for i in range(3)]
        bad = dict(reqs[1], N=p.N - 2)  # another ensemble size than the batch's
        with pytest.raises(oic.OicError) as e:
            grp.solve([(0, reqs[0]), (1, bad), (2, reqs[2])])
        assert e.value.code == oic.OIC_EINVAL
        assert grp.rc_codes == [0, oic.OIC_EINVAL, 0]
        # the others ran (their results are written where solve() put them: re-run to read)
        outs = grp.solve([(0, reqs[0]), (2, reqs[2])])
        assert np.array_equal(outs[0][0], alone[0][0]) and np.array_equal(outs[1][0], alone[2][0])
        with pytest.raises(oic.OicError):
            grp.solve([(0, reqs[0]), (0, reqs[0])])  # a slot twice


def test_group_rejects_configurations_without_grouped_kernels():
    p = FAMILIES["c16_ragged"]
    with pytest.raises(oic.OicError):
        oic.Group(p.n, p.m, p.l, p.channels, p.activation, p.N, p.H, 2, precision=oic.OIC_PREC_FP32)
    # one slot takes any configuration: its batch is its own solve
    prob = _problems(p, 1)[0]
    with oic.Group(p.n, p.m, p.l, p.channels, p.activation, p.N, p.H, 1, precision=oic.OIC_PREC_FP32) as grp:
        grp.slots[0].set_weights(prob.B, prob.weights)
        req = _request(prob, 0)
        U, X = grp.solve([(0, req)])[0]
        with oic.Controller(p.n, p.m, p.l, p.channels, p.activation, p.N, p.H) as c:
            c.set_weights(prob.B, prob.weights)
            Uc, Xc = c.solve_ex(**req)
        assert np.array_equal(U, Uc) and np.array_equal(X, Xc)


def test_new_weights_in_a_slot_reach_the_captured_grouped_solve():
    """The captured grouped solve holds buffer addresses, not contents: after new weights
    (and a bias switched on) are copied into a slot, the next batch uses them, bitwise as
    the slot's own solve with the new weights."""
    p = FAMILIES["c32"]
    probs = _problems(p, 3)
    with oic.Group(p.n, p.m, p.l, p.channels, p.activation, p.N, p.H, 2) as grp:
        for i in range(2):
            grp.slots[i].set_weights(probs[i].B, probs[i].weights)
        reqs = [_request(probs[i], i) for i in range(2)]
        grp.solve([(0, reqs[0]), (1, reqs[1])])  # captures the grouped solve
        grp.slots[1].set_weights(probs[2].B, probs[2].weights, _biases(probs[2], 9))
        alone = grp.slots[1].solve_ex(**reqs[1])
        outs = grp.solve([(0, reqs[0]), (1, reqs[1])])
        assert np.array_equal(outs[1][0], alone[0]) and np.array_equal(outs[1][1], alone[1])
        with oic.Controller(p.n, p.m, p.l, p.channels, p.activation, p.N, p.H,
                            precision=oic.OIC_PREC_BF16) as c:
            c.set_weights(probs[2].B, probs[2].weights, _biases(probs[2], 9))
            U, X = c.solve_ex(**reqs[1])
        assert np.array_equal(U, alone[0]) and np.array_equal(X, alone[1])


def test_device_memory_group_matches_host_memory_group():
    """A group created for device memory (torch tensors in and out, its work ordered on the
    caller's stream) gives the host-memory group's results bitwise."""
    import torch
    p = FAMILIES["c16_ragged"]
    probs = _problems(p, 2)
    reqs = [_request(pr, i) for i, pr in enumerate(probs)]
    with oic.Group(p.n, p.m, p.l, p.channels, p.activation, p.N, p.H, 2) as grp:
        for i, pr in enumerate(probs):
            grp.slots[i].set_weights(pr.B, pr.weights)
        host = grp.solve([(0, reqs[0]), (1, reqs[1])])
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    dreqs = [dict(r, X0=dev(r["X0"]), reference=dev(r["reference"]), U_prev=dev(r["U_prev"])) for r in reqs]
    with oic.Group(p.n, p.m, p.l, p.channels, p.activation, p.N, p.H, 2, mem_mode=oic.OIC_MEM_DEVICE) as grp:
        for i, pr in enumerate(probs):
            grp.slots[i].set_weights(pr.B, pr.weights)
        outs = grp.solve([(0, dreqs[0]), (1, dreqs[1])])
        torch.cuda.synchronize()
        for (U, X), (Uh, Xh) in zip(outs, host):
            assert np.array_equal(U.cpu().numpy(), Uh) and np.array_equal(X.cpu().numpy(), Xh)


def test_dense_noise_factors_in_a_batch():
    """Requests with dense Q and R (their Cholesky factors drive the noise as full
    triangles) batch together like diagonal ones, bitwise as each slot's own solve; a
    request whose factor layout differs from the batch's fails alone."""
    p = FAMILIES["c16_ragged"]
    probs = _problems(p, 3)
    dense = [dict(Q=wl.random_spd(p.l, 50 + i, scale=0.05), R=wl.random_spd(p.n, 60 + i, scale=0.005))
             for i in range(3)]
    with oic.Group(p.n, p.m, p.l, p.channels, p.activation, p.N, p.H, 3) as grp:
        for i, pr in enumerate(probs):
            grp.slots[i].set_weights(pr.B, pr.weights)
        reqs = [dict(_request(pr, i), **dense[i]) for i, pr in enumerate(probs)]
        alone = [grp.slots[i].solve_ex(**reqs[i]) for i in range(3)]
        outs = grp.solve([(i, reqs[i]) for i in range(3)])
        for i in range(3):
            assert np.array_equal(outs[i][0], alone[i][0]) and np.array_equal(outs[i][1], alone[i][1]), i
        # slot 1 back to diagonal factors: the batch takes slot 0's dense layout, slot 1 fails
        mixed = [reqs[0], _request(probs[1], 1), reqs[2]]
        with pytest.raises(oic.OicError):
            grp.solve([(i, mixed[i]) for i in range(3)])
        assert grp.rc_codes == [0, oic.OIC_EINVAL, 0]


def test_a_slot_with_a_constraint_fails_alone_and_solves_on_its_own():
    """A constraint adds an observation row that the grouped kernels do not carry: a slot
    with one set fails in a batch (the others run), still solves on its own, and joins
    batches again once the constraint is removed."""
    p = FAMILIES["c16_ragged"]
    probs = _problems(p, 2)
    with oic.Group(p.n, p.m, p.l, p.channels, p.activation, p.N, p.H, 2) as grp:
        for i, pr in enumerate(probs):
            grp.slots[i].set_weights(pr.B, pr.weights)
        reqs = [_request(pr, i) for i, pr in enumerate(probs)]
        alone = [grp.slots[i].solve_ex(**reqs[i]) for i in range(2)]
        grp.slots[1].set_constraint(np.full(p.n, 0.1, np.float32), np.full(p.l, 0.2, np.float32), b=1.0)
        with pytest.raises(oic.OicError):
            grp.solve([(0, reqs[0]), (1, reqs[1])])
        assert grp.rc_codes == [0, oic.OIC_EINVAL]
        constrained = grp.slots[1].solve_ex(**reqs[1])
        assert not np.array_equal(constrained[0], alone[1][0])
        grp.slots[1].set_constraint()
        outs = grp.solve([(0, reqs[0]), (1, reqs[1])])
        for i in range(2):
            assert np.array_equal(outs[i][0], alone[i][0]) and np.array_equal(outs[i][1], alone[i][1]), i
