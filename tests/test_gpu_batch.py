"""GPU tests of the batched path (lbm_batch_* of the C ABI): many lattices of
different sizes and wall rules advanced by one launch per time step.

A member's state must be bit for bit the state lbm_step gives the same lattice
alone (both run the same per-node arithmetic), whatever else is in the batch,
whatever the block size and whether the steps are replayed from a HIP graph;
its residuals depend on nothing but itself and the block size.  FP64 members
are also checked against the oracle."""
import sys

import numpy as np
import pytest

import lbm_inputs
import oracle
from lbm_inputs import face

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from paper_1611_03329_amd import Batch, Lattice, LBMError  # noqa: E402

WALL = face("wall", "adiabatic")
PER = face("periodic", "periodic")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _members():
    """Seven D3Q19 workloads: four with the lean wall rules (static walls,
    periodic faces), three with the general ones (a moving lid; an inlet and
    an open outlet, twice); two of them have separable tiles.  Name ->
    (workload, random-state seed or None)."""
    lid = lbm_inputs.cavity((13, 7, 5), porosity=0.55, darcy=5e-3, rayleigh=2e5)
    lid["faces"] = [face("wall", "isothermal", 0.5), face("wall", "isothermal", -0.5), WALL, WALL,
                    WALL, face("wall", "adiabatic", 0.0, (0.02, -0.01, 0.0))]
    perx = lbm_inputs.cavity((11, 6, 9), porosity=0.55, darcy=5e-3, rayleigh=2e5)
    perx["faces"] = [PER, PER, face("wall", "isothermal", 0.3), face("wall", "isothermal", -0.2), WALL, WALL]
    return {
        "cavity": (lbm_inputs.cavity((12, 10, 9), rayleigh=5e4, seed=4), None),
        "lid": (lid, 11),
        "perx": (perx, 12),
        "channel": (lbm_inputs.channel((16, 8, 6), lattice=19), None),
        # separable tiles (64 divides the 2048-node tile, 32 rows per tile divide
        # ny): in FP16 mode these take the odd-step kernel with per-axis link
        # deltas, a launch group of their own
        "sep": (lbm_inputs.cavity((64, 32, 3), rayleigh=1e5, seed=8), 13),
        "sepchan": (lbm_inputs.channel((64, 32, 4), lattice=19), None),
        # more tiles than a persistent grid of 1 block/CU at 256 threads or
        # 4 blocks/CU at 64 threads has blocks: those blocks take several tiles
        "big": (lbm_inputs.cavity((48, 47, 49), rayleigh=1e5, seed=6), None),
    }


def _make(wl, seed, prec, check):
    lat = Lattice(wl, prec, check_interval=check)
    if seed is not None:
        f0, g0 = lbm_inputs.random_state(wl["q"], lat.shape, seed, amp=0.05, T_amp=0.4)
        lat.set_state(f0, g0)
    return lat


def _state(lat):
    f, g = lat.get_state()
    lat.stream.synchronize()
    torch.cuda.synchronize()
    return f, g


def _same(a, b):
    fa, ga = _state(a)
    fb, gb = _state(b)
    return torch.equal(fa, fb) and torch.equal(ga, gb)


MiB = 1 << 20


@pytest.mark.parametrize("prec,block,per_cu,group,xcd", [
    ("fp64", 256, 0, 0, 0), ("fp32", 64, 0, 0, 0), ("fp16", 128, 0, 0, 0), ("fp32", 256, 1, 0, 0),
    ("fp16", 64, 4, 0, 0), ("fp32", 256, 0, MiB, 0), ("fp64", 128, 4, 2 * MiB, 0), ("fp32", 256, 0, MiB, 8),
    ("fp16", 64, 1, 0, 8), ("fp32", 128, 0, 0, 3)])
def test_batch_members_match_solo_bitwise(prec, block, per_cu, group, xcd):
    """Each member of a mixed batch (lean and general wall rules, five sizes)
    equals the same lattice stepped alone, bit for bit, at both parities: with
    one block per tile or a persistent grid (per_cu > 0), in hardware tile
    order or in contiguous per-XCD ranges, and with the members in one group
    per wall-rule set or split into groups of at most `group` bytes that run
    whole check intervals one after another."""
    _say(f"case batch-vs-solo {prec} block {block} per_cu {per_cu} group {group} xcd {xcd}")
    ms = _members()
    solo = {k: _make(wl, sd, prec, 0) for k, (wl, sd) in ms.items()}
    with Batch(check_interval=6, block=block, per_cu=per_cu, group_bytes=group, xcd_ranges=xcd) as b:
        mem = {k: _make(wl, sd, prec, 0) for k, (wl, sd) in ms.items()}
        for k in ms:
            b.add(mem[k])
        for n in (1, 4, 13):
            b.step(n)
            for k in ms:
                solo[k].step(n)
            for k in ms:
                assert mem[k].time == solo[k].time
                assert _same(mem[k], solo[k]), (k, solo[k].time)
        for m in list(mem.values()):
            m.close()
    for s in solo.values():
        s.close()


def _theta_residual(a, b, wl):
    """r(n) from fields at n-1 (a) and n (b), straight from its definition."""
    du = np.sqrt(sum(np.sum((b[k] - a[k]) ** 2) for k in ("ux", "uy", "uz")))
    un = np.sqrt(sum(np.sum(b[k] ** 2) for k in ("ux", "uy", "uz")))
    ta = (a["T"] - wl["T_ref"]) / wl["delta_T"] + 0.5
    tb = (b["T"] - wl["T_ref"]) / wl["delta_T"] + 0.5
    return max(du / un, np.sqrt(np.sum((tb - ta) ** 2)) / np.sqrt(np.sum(tb ** 2)))


def test_batch_fp64_matches_oracle():
    """FP64 members against the oracle: states to 1e-12 after 9 steps and the
    batch residual r(8) (snapshot at batch step 7, compare at 8) against the
    definition applied to oracle fields at 7 and 8."""
    _say("case batch fp64 vs oracle, K=4, 9 steps")
    ms = _members()
    refs = {}
    for k, (wl, sd) in ms.items():
        with oracle.Oracle(wl) as o:
            if sd is not None:
                f0, g0 = lbm_inputs.random_state(wl["q"], o.shape, sd, amp=0.05, T_amp=0.4)
                o.set_state(f0, g0)
            o.step(7)
            a = o.fields()
            o.step(1)
            bf = o.fields()
            o.step(1)
            refs[k] = (_theta_residual(a, bf, wl), o.get_state())
    with Batch(check_interval=4) as b:
        mem = {k: _make(wl, sd, "fp64", 0) for k, (wl, sd) in ms.items()}
        for k in ms:
            b.add(mem[k])
        b.step(9)
        r, at, un = b.residuals()
        for i, k in enumerate(ms):
            assert at[i] == 8 and not un[i], (k, at[i], un[i])
            assert abs(r[i] - refs[k][0]) <= 1e-8 * refs[k][0], (k, r[i], refs[k][0])
            f, g = _state(mem[k])
            fr, gr = refs[k][1]
            assert np.max(np.abs(f.cpu().numpy() - fr)) <= 1e-12 * np.max(np.abs(fr)), k
            assert np.max(np.abs(g.cpu().numpy() - gr)) <= 1e-12 * np.max(np.abs(gr)), k
            # the member's own query sees the batch's check
            rr, aa = mem[k].residual()
            assert aa == 8 and rr == r[i]
        for m in list(mem.values()):
            m.close()


def test_alone_vs_mix_results_are_identical():
    """A lattice alone in a batch and the same lattice in a batch with three
    others give identical states and identical residuals (bitwise)."""
    _say("case alone-vs-mix fp32 K=5 block 128")
    ms = _members()
    wl, sd = ms["lid"]
    with Batch(check_interval=5, block=128) as alone, Batch(check_interval=5, block=128) as mix:
        a = _make(wl, sd, "fp32", 0)
        alone.add(a)
        others = [_make(w, s, "fp32", 0) for k, (w, s) in ms.items() if k != "lid"]
        m = _make(wl, sd, "fp32", 0)
        mix.add(others[0])
        mix.add(m)
        mix.add(others[1])
        mix.add(others[2])
        mix.add(others[3])
        for n in (3, 7, 11):
            alone.step(n)
            mix.step(n)
            assert _same(a, m)
            ra, ta, _ = alone.residuals()
            rm, tm, _ = mix.residuals()
            assert ta[0] == tm[1] and ra[0] == rm[1], (ra, rm)
        assert ta[0] == 20
        for x in [a, m] + others:
            x.close()


def test_join_and_leave_mid_schedule():
    """A lattice that joins at an odd batch step (parity differs: it takes one
    step of its own) and one that leaves keep the solo trajectory; the joiner's
    first check comes after its first snapshot inside the batch."""
    _say("case join/leave fp64 K=4")
    ms = _members()
    with Batch(check_interval=4) as b:
        stay = _make(*ms["cavity"], "fp64", 0)
        leave = _make(*ms["lid"], "fp64", 0)
        b.add(stay)
        b.add(leave)
        b.step(7)                       # batch s = 7, parity odd
        join = _make(*ms["perx"], "fp64", 0)
        b.add(join)                     # one solo step: join.time == 1
        assert join.time == 1
        b.step(2)                       # snapshot at s = 7 (the joiner's first), compare at s = 8
        r, at, _ = b.residuals()
        assert at == [8, 8, 2], at
        b.remove(leave)
        leave.step(5)                   # a plain lattice again
        b.step(4)                       # s = 13: snapshot at 11, compare at 12
        r, at, _ = b.residuals()
        assert at == [12, join.time - 1], at
        assert len(b) == 2
        ref_s = _make(*ms["cavity"], "fp64", 0)
        ref_l = _make(*ms["lid"], "fp64", 0)
        ref_j = _make(*ms["perx"], "fp64", 0)
        ref_s.step(13)
        ref_l.step(14)
        ref_j.step(7)
        assert stay.time == 13 and leave.time == 14 and join.time == 7
        assert _same(stay, ref_s) and _same(leave, ref_l) and _same(join, ref_j)
        # a member cannot be stepped alone
        with pytest.raises(LBMError):
            join.step(1)
        join.close()                    # leaves the batch first
        assert len(b) == 1
        for x in (stay, leave, ref_s, ref_l, ref_j):
            x.close()


@pytest.mark.parametrize("group", [0, MiB])
def test_graph_replay_matches_eager(group):
    """Check intervals replayed from a HIP graph give the eager results on every
    replay, with eager work and synchronizations between the replays."""
    _say(f"case graph replay fp32 K=8 group {group}")
    ms = _members()
    with Batch(check_interval=8, graph=True, group_bytes=group) as gb, Batch(check_interval=8) as eb:
        g = {k: _make(w, s, "fp32", 0) for k, (w, s) in ms.items()}
        e = {k: _make(w, s, "fp32", 0) for k, (w, s) in ms.items()}
        for k in ms:
            gb.add(g[k])
            eb.add(e[k])
        gb.step(8)
        eb.step(8)
        for rep in range(4):
            gb.step(8)                  # one replay
            eb.step(8)
            torch.cuda.synchronize()
            x = torch.ones(1 << 20, device="cuda").sum()  # unrelated eager work
            assert float(x) == float(1 << 20)
            for k in ms:
                assert _same(g[k], e[k]), (rep, k)
            rg, tg, _ = gb.residuals()
            re, te, _ = eb.residuals()
            assert rg == re and tg == te, (rep, rg, re)
        gb.step(3)                      # a partial chunk runs eagerly
        eb.step(3)
        for k in ms:
            assert _same(g[k], e[k]), k
        for x in list(g.values()) + list(e.values()):
            x.close()


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_size_class_tiles_keep_results(prec):
    """Members of different size classes on different tile sizes (64 threads
    for the smallest classes, 128 for the middle ones, the batch's 256 for the
    rest) launch in separate groups and still equal their solo states bit for
    bit, at both parities."""
    _say(f"case size-class tiles {prec}")
    ms = _members()
    solo = {k: _make(wl, sd, prec, 0) for k, (wl, sd) in ms.items()}
    with Batch(check_interval=6) as b:
        for k_, blk in ((8, 64), (9, 64), (10, 128), (12, 128)):
            b.set_class_block(k_, blk)
        mem = {k: _make(wl, sd, prec, 0) for k, (wl, sd) in ms.items()}
        for k in ms:
            b.add(mem[k])
        assert b.class_blocks() == {8: 64, 9: 64, 10: 128, 12: 128}
        for n in (1, 4, 13):
            b.step(n)
            for k in ms:
                solo[k].step(n)
            for k in ms:
                assert _same(mem[k], solo[k]), (k, solo[k].time)
        for m in list(mem.values()):
            m.close()
    for x in solo.values():
        x.close()


def test_autotune_keeps_results():
    """The autotuner picks one of the admissible launch shapes; the steps it
    takes are ordinary steps (the state still equals the solo state)."""
    _say("case autotune fp32")
    ms = _members()
    with Batch(check_interval=10) as b:
        mem = {k: _make(w, s, "fp32", 0) for k, (w, s) in ms.items()}
        for k in ms:
            b.add(mem[k])
        block, per_cu, group, xcd = b.autotune()
        assert block in (64, 128, 256) and per_cu in (0, 4, 8) and xcd in (0, 8)
        assert group in [0] + [m * MiB for m in (8, 16, 32, 64, 128, 256, 512)]
        classes = {int(np.floor(np.log2(m.nodes))) for m in mem.values()}
        tuned = b.class_blocks()
        assert set(tuned) <= classes and set(tuned.values()) <= {64, 128, 256}
        b.step(4)
        steps = mem["cavity"].time
        # 16 group/order pairs + 2 tile sizes + 2 grids + 2 tile sizes per size
        # class, four intervals each (one untimed, three timed)
        assert steps == (16 + 2 + 2 + 2 * len(classes)) * 4 * 10 + 4
        for k, (w, s) in ms.items():
            ref = _make(w, s, "fp32", 0)
            ref.step(steps)
            assert _same(mem[k], ref), k
            ref.close()
        for m in list(mem.values()):
            m.close()


def test_unstable_member_does_not_disturb_the_others():
    """A member with a NaN is flagged at the next check; the other members'
    states still equal their solo states."""
    _say("case unstable member fp64 K=3")
    ms = _members()
    with Batch(check_interval=3) as b:
        bad = _make(*ms["cavity"], "fp64", 0)
        f, g = _state(bad)
        f[3, 5, 5, 5] = float("nan")
        bad.set_state(f, g)
        good = _make(*ms["channel"], "fp64", 0)
        b.add(bad)
        b.add(good)
        b.step(7)
        r, at, un = b.residuals()
        assert un == [True, False], un
        b.remove(bad)
        ref = _make(*ms["channel"], "fp64", 0)
        ref.step(7)
        assert _same(good, ref)
        for x in (bad, good, ref):
            x.close()


def test_batch_rejects_mixed_precision_and_bad_block():
    ms = _members()
    with Batch(check_interval=4) as b:
        a = _make(*ms["cavity"], "fp32", 0)
        c = _make(*ms["cavity"], "fp64", 0)
        b.add(a)
        with pytest.raises(LBMError):
            b.add(c)
        with pytest.raises(LBMError):
            b.set_launch(96)
        with pytest.raises(LBMError):
            b.set_launch(128, -1)
        with pytest.raises(LBMError):
            b.set_launch(128, 0, 0, -2)
        with pytest.raises(LBMError):
            b.add(a)
        a.close()
        c.close()


@pytest.mark.parametrize("src_prec,dst_prec", [("fp16", "fp32"), ("fp32", "fp64"), ("fp32", "fp32")])
def test_transfer_state_converts_precision(src_prec, dst_prec):
    """lbm_transfer_state copies the logical state across precisions (from an
    odd time, i.e. the other storage parity): the destination's state equals
    the source's exactly (every value is representable), and an FP32 copy of
    an FP32 lattice continues on the same trajectory."""
    _say(f"case transfer {src_prec} -> {dst_prec}")
    wl, sd = _members()["big"]
    src = _make(wl, sd, src_prec, 0)
    src.step(5)
    dst = _make(wl, sd, dst_prec, 0)
    dst.transfer_from(src)
    fs, gs = _state(src)
    fd, gd = _state(dst)
    assert torch.equal(fs, fd) and torch.equal(gs, gd)
    if src_prec == dst_prec:
        src.step(6)
        dst.step(6)
        fs, gs = _state(src)
        fd, gd = _state(dst)
        assert torch.allclose(fd, fs, rtol=1e-6, atol=0) and torch.allclose(gd, gs, rtol=1e-6, atol=1e-9)
    src.close()
    dst.close()


def test_span_residual_matches_oracle():
    """With the span residual the check at step 8 (interval 4) compares the
    state with that of step 4: r equals the definition applied to oracle
    fields at 4 and 8.  Graph replay and group size do not change it."""
    _say("case span residual fp64 K=4")
    wl, sd = _members()["lid"]
    with oracle.Oracle(wl) as o:
        f0, g0 = lbm_inputs.random_state(wl["q"], o.shape, sd, amp=0.05, T_amp=0.4)
        o.set_state(f0, g0)
        o.step(4)
        a = o.fields()
        o.step(4)
        r_ref = _theta_residual(a, o.fields(), wl)
    out = []
    for graph in (False, True):
        with Batch(check_interval=4, span=True, graph=graph) as b:
            lat = _make(wl, sd, "fp64", 0)
            b.add(lat)
            b.step(9)
            r, at, un = b.residuals()
            assert at == [8] and not un[0]
            assert abs(r[0] - r_ref) <= 1e-9 * r_ref, (r[0], r_ref)
            out.append(r[0])
            lat.close()
    assert out[0] == out[1]


@pytest.mark.parametrize("prec,shape", [("fp32", (256, 128, 128)), ("fp64", (256, 128, 128)),
                                        ("fp16", (256, 256, 128))])
def test_capped_even_step_changes_no_state(prec, shape):
    """A lean lattice large enough for the even step's residency cap (lbm_step
    launches its plain even steps with two resident blocks per CU, four for
    FP16 storage) ends bit for bit where its one-member batch (launches
    uncapped) does, over steps of both parities and a residual check."""
    wl = lbm_inputs.cavity(shape, porosity=0.5, darcy=1e-3, rayleigh=1e5, seed=17)
    _say(f"case capped even step vs batch launch {prec} {shape}")
    solo = _make(wl, None, prec, 4)
    solo.step(9)
    with Batch(check_interval=4) as b:
        mem = _make(wl, None, prec, 4)
        b.add(mem)
        b.step(9)
        assert _same(solo, mem)
        b.remove(mem)
    mem.close()
    solo.close()
