"""Host emulation of the direct-load rings' schedule (the rotation's K loop,
the grid ring kernel's passes): randomised timings of several waves that run
the kernels' step sequence, with the hardware rules the protocol relies on,
checking that no wave reads an LDS slot or a register set before every load
of its step has landed, and that no load lands in a slot or register set
while a wave may still read what it replaces.

Rules modelled: a wave's vector-memory loads (global-to-LDS and into
registers) complete in issue order, each after an arbitrary delay; `s_waitcnt
vmcnt(N)` blocks the wave until at most N of its loads are outstanding;
`s_waitcnt lgkmcnt(0); s_barrier` (lds_barrier) waits for the wave's own LDS
reads, then for every wave to arrive.  The step sequence restated from the
kernels (a change there must be mirrored here): issue slots 0 and 1 (steps 0
and 1); for step s: wait until the loads of step s + 1 alone are outstanding,
barrier, issue step s + 2 (clamped to the last step) into slot (s + 2) % R,
read slot s % R; after the last step wait for every load and barrier (the
epilogue then reuses the ring).  R = 3 slots (R = 4 for the four-slot
rotation ring: waits leave R - 2 steps outstanding, issues go R - 1 ahead)."""
import numpy as np
import pytest


def emulate(n_waves, n_steps, lds_per_step, reg_per_step, ring, rng, mistake=None):
    """One randomised run; returns the violations found (empty when safe).
    `mistake` plants an error in the protocol (for the test that the checks
    can fail): "wait" leaves one more step outstanding at the wait, "barrier"
    drops the barrier, "ahead" issues one step further ahead."""
    ahead = ring - 1 + (mistake == "ahead")  # steps issued ahead of the one read
    per_step = lds_per_step + reg_per_step
    bad = []
    # per wave: list of (complete_time, kind, slot, step) in issue order
    loads = [[] for _ in range(n_waves)]
    t = np.zeros(n_waves)                 # each wave's clock
    last_done = np.zeros(n_waves)         # in-order completion: a load ends no earlier than the one before
    # slot writes: slot -> list of (land_time, step); reads: slot -> list of (start, end, step, wave)
    writes = {u: [] for u in range(ring)}
    reads = {u: [] for u in range(ring)}
    rwrites = [{u: [] for u in range(ring)} for _ in range(n_waves)]
    rreads = [{u: [] for u in range(ring)} for _ in range(n_waves)]

    def issue(w, step):
        s = min(step, n_steps - 1)        # past the last step the loads repeat it into a slot not read again
        u = step % ring
        for q in range(per_step):
            t[w] += rng.uniform(0.1, 1.0)
            done = max(last_done[w], t[w] + rng.exponential(20.0) + rng.uniform(0, 5))
            last_done[w] = done
            kind = "lds" if q < lds_per_step else "reg"
            loads[w].append((done, kind, u, step))
            (writes[u] if kind == "lds" else rwrites[w][u]).append((done, step))

    def wait_vm(w, n_out):
        # block until at most n_out of this wave's loads are outstanding
        pend = sorted(d for d, *_ in loads[w] if d > t[w])
        if len(pend) > n_out:
            t[w] = max(t[w], pend[len(pend) - n_out - 1])

    def barrier():
        if mistake == "barrier":
            return
        tb = t.max() + rng.uniform(0.0, 2.0)
        t[:] = tb

    for w in range(n_waves):
        for j in range(ahead):
            issue(w, j)
    read_start = {}
    for s in range(n_steps):
        for w in range(n_waves):
            t[w] += rng.uniform(0, 3)
            wait_vm(w, (ring - 2 + (mistake == "wait")) * per_step)
        barrier()
        # reads of the previous step ended before this barrier (lgkmcnt(0) before s_barrier)
        for w in range(n_waves):
            if s > 0:
                u0, st0, s0 = read_start[w]
                reads[u0].append((st0, t[w], s0, w))
                rreads[w][u0].append((st0, t[w], s0))
        for w in range(n_waves):
            issue(w, s + ahead)
            t[w] += rng.uniform(0, 3)
            read_start[w] = (s % ring, t[w], s)
            t[w] += rng.uniform(5, 40)    # the multiply-accumulate work of the step
    for w in range(n_waves):
        wait_vm(w, 0)
    barrier()
    for w in range(n_waves):
        u0, st0, s0 = read_start[w]
        reads[u0].append((st0, t[w], s0, w))
        rreads[w][u0].append((st0, t[w], s0))
    t_end = t.max()
    # LDS: every load of step s into slot u (all waves) lands before any read of step s starts;
    # no load of a later step into u lands before every read of an earlier step of u has ended
    for u in range(ring):
        for (st0, en0, s0, w) in reads[u]:
            for (land, ws) in writes[u]:
                if ws == s0 and land > st0:
                    bad.append(("lds read before its data", u, s0, w))
                if ws > s0 and land < en0 and ws < n_steps + ahead:
                    bad.append(("lds overwritten while read", u, s0, ws, w))
    # registers: the same per wave (a set is read by the wave that loaded it)
    for w in range(n_waves):
        for u in range(ring):
            for (st0, en0, s0) in rreads[w][u]:
                for (land, ws) in rwrites[w][u]:
                    if ws == s0 and land > st0:
                        bad.append(("register read before its data", u, s0, w))
                    if ws > s0 and land < en0:
                        bad.append(("register overwritten while read", u, s0, ws, w))
    # nothing in flight once the ring is handed to the epilogue
    for w in range(n_waves):
        if any(d > t_end for d, *_ in loads[w]):
            bad.append(("load in flight after the loop", w))
    return bad


CASES = [  # (name, waves, steps, LDS loads per wave per step, register loads, ring slots)
    ("rotation 64x256, three slots", 8, 16, 4, 0, 3),
    ("rotation 64x128, three slots", 4, 5, 8, 0, 3),
    ("rotation 64x256, four slots", 8, 7, 4, 0, 4),
    ("rotation, one step", 4, 1, 8, 0, 3),
    ("rotation, two steps", 4, 2, 8, 0, 3),
    ("grid pass A (two slices a step)", 4, 16, 2, 8, 3),
    ("grid pass B", 4, 32, 4, 4, 3),
    ("grid one pass, p_L = 2", 4, 8, 4, 8, 3),
    ("grid, four steps", 4, 4, 4, 4, 3),
]


@pytest.mark.parametrize("name,waves,steps,lpw,xpw,ring", CASES)
def test_ring_schedule_is_safe(name, waves, steps, lpw, xpw, ring):
    rng = np.random.default_rng(2024)
    for trial in range(60):
        bad = emulate(waves, steps, lpw, xpw, ring, rng)
        assert not bad, (name, trial, bad[:3])


@pytest.mark.parametrize("mistake", ["wait", "barrier", "ahead"])
def test_emulation_catches_a_planted_mistake(mistake):
    """The emulation is not vacuous: with the wait before the barrier leaving
    one more step of loads in flight, with the barrier dropped, or with the
    loads issued one step further ahead than the ring has slots for, it finds
    slots read before their data has landed or overwritten while read."""
    rng = np.random.default_rng(7)
    found = False
    for trial in range(40):
        found = found or bool(emulate(4, 12, 4, 4, 3, rng, mistake=mistake))
    assert found
