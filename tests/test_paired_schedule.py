"""The launch schedule of the paired propagator sweeps, checked on the host.

The evaluation with paired kernels (tiles with k = -1) runs N launches, launch j taking
forward step j and backward step N + 1 + (N mod 2) - j when that lies in 2..N, then
backward step 1 alone; for even N >= 4 backward step N has no launch (launch 1 takes none)
and backward step N - 1 forms G+_N from bead N's stored field factor.  Below the crossing
se = (N + N mod 2) / 2 the forward step of a bead runs first and stores G_s in slot s - 1;
above it the backward step runs first and stores sigma_s there.  The flags below are the
ones the evaluation computes for each launch (f_late, f_from_pp, f_to_pp, g_late, g_exp,
g_from_e), read from the library's host function that the evaluation itself calls.  This test replays the schedule over symbolic
buffers and checks, for every N the library takes, that no launch writes a buffer that
another workgroup of the same launch reads (through the stencil, or from the other half),
and that every read sees the value the step needs."""
import pytest


def launches(N):
    """The library's own schedule (hsf_paired_schedule, host code, no GPU)."""
    import ctypes
    from paper_1204_2088_amd import hsf
    lib = hsf.load()
    out = []
    for j in range(1, N + 1):
        v = (ctypes.c_int * 8)()
        assert lib.hsf_paired_schedule(N, j, v) == hsf.HSF_OK
        out.append(dict(sf=v[0], sb=v[1], f_late=bool(v[2]), f_from_pp=bool(v[3]), f_to_pp=bool(v[4]),
                        g_late=bool(v[5]), g_exp=bool(v[6]), g_from_e=bool(v[7])))
    return out


def test_schedule_arguments_are_checked():
    import ctypes
    from paper_1204_2088_amd import hsf
    lib = hsf.load()
    v = (ctypes.c_int * 8)()
    for N, j in ((1, 1), (65, 1), (8, 0), (8, 9)):
        assert lib.hsf_paired_schedule(N, j, v) == hsf.HSF_EINVAL


def replay(N):
    """Accesses per launch: (half, buffer, mode) with mode 's' (stencil read), 'r' (own
    site read) or 'w' (write); expected contents of every read."""
    ops = []
    par = 0
    for L in launches(N):
        acc, reads, writes = [], [], []
        s = L["sf"]
        if s == 1:
            writes.append(("f", "E", "E"))
        else:
            src = ("fpp", (s - 1) % 2) if L["f_from_pp"] else ("slot", s - 2)
            acc.append(("f", src, "s")); reads.append((src, ("G", s - 1)))
            acc.append(("f", "E", "r")); reads.append(("E", "E"))
        if L["f_late"]:
            if s < N:
                acc.append(("f", ("slot", s - 1), "r")); reads.append((("slot", s - 1), ("sigma", s)))
            writes.append(("f", ("slot", s - 1), ("term", s)))
        else:
            writes.append(("f", ("slot", s - 1), ("G", s)))
        if L["f_to_pp"]:
            writes.append(("f", ("fpp", s % 2), ("G", s)))
        sb = L["sb"]
        if sb:
            gin, gout = ("Gp", par ^ 1), ("Gp", par)
            par ^= 1
            if L["g_from_e"]:   # G+_N from bead N's field factor, stored by forward step 1
                assert sb == N - 1
                acc.append(("b", "E", "s")); reads.append(("E", "E"))
            elif sb < N:
                acc.append(("b", gin, "s")); reads.append((gin, ("G+", sb + 1)))
            if not L["g_exp"]:
                acc.append(("b", "E", "r")); reads.append(("E", "E"))
            writes.append(("b", gout, ("G+", sb)))
            if L["g_late"]:
                acc.append(("b", ("slot", sb - 1), "r")); reads.append((("slot", sb - 1), ("G", sb)))
                writes.append(("b", ("slot", sb - 1), ("term", sb)))
            elif sb < N:
                writes.append(("b", ("slot", sb - 1), ("sigma", sb)))
        acc += [(h, b, "w") for h, b, _ in writes]
        ops.append((acc, reads, [(b, v) for _, b, v in writes]))
    # backward step 1, alone: stencil of G+_2, G_1 and the terms of steps 2..N
    gin = ("Gp", par ^ 1)
    reads = [(gin, ("G+", 2)), (("slot", 0), ("G", 1))] + [(("slot", k), ("term", k + 1)) for k in range(1, N)]
    ops.append(([], reads, []))
    return ops


@pytest.mark.parametrize("N", range(2, 65))
def test_paired_schedule_is_race_free_and_complete(N):
    state = {}
    steps_f, steps_b = set(), set()
    for L in launches(N):
        steps_f.add(L["sf"])
        if L["sb"]:
            steps_b.add(L["sb"])
    folded = N % 2 == 0 and N >= 4   # backward step N formed inside step N - 1
    assert steps_f == set(range(1, N + 1)) and steps_b == set(range(2, N if folded else N + 1))
    assert sum(L["g_from_e"] for L in launches(N)) == (1 if folded else 0)
    for acc, reads, writes in replay(N):
        by = {}
        for h, b, m in acc:
            by.setdefault(b, []).append((h, m))
        for b, lst in by.items():
            ws = {h for h, m in lst if m == "w"}
            assert len(ws) <= 1, (N, b, lst)                      # one half writes a buffer
            for h, m in lst:
                if ws and m == "s":
                    assert False, (N, b, "stencil read of a buffer written in the same launch")
                if ws and m == "r":
                    assert h in ws, (N, b, "own-site read from the other half's writes")
        for b, want in reads:
            assert state.get(b) == want, (N, b, want, state.get(b))
        for b, v in writes:
            state[b] = v


def test_paired_schedule_launch_count():
    for N in range(2, 65):
        assert len(launches(N)) + 1 == N + 1
