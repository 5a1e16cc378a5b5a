"""Host model of the X-engine's DMA stage schedule (xtile_mm16 in
paper_1609_04205_amd/csrc/xengine.hip): for every block count, stage size
and depth, each stage is issued exactly once, and the loads the kernel
issues with an unclamped (scalar, not range-checked) stage offset cover
whole blocks of the channel's data only.  The model follows the kernel's
control flow: the prologue, the main loop of RS-stage groups, the group that
loads the final group's first stage, and the final group; tiles with the
column-register ring (RS = depth + 1) skip the clamp in the main loop,
tiles without it (RS = 1) always clamp."""
import pytest


def schedule(nb, k_stg, depth, ring):
    rs = depth + 1 if ring else 1
    n_st = -(-nb // (k_stg * rs)) * rs
    n_final = n_st - rs
    issued = []

    def issue(s, clamp):
        assert 0 <= s < n_st
        if not clamp:
            assert (s + 1) * k_stg <= nb, f"stage {s} issued unclamped past the {nb} blocks"
        issued.append(s)

    for d in range(depth):
        if ring or d < n_st:
            issue(d, True)
    if ring or depth < n_st:
        issue(depth, True)

    def stage(s, has_next, final, clamp):
        if not has_next:
            return
        t = s + 1 + depth
        if ring:
            if not final:
                issue(t, clamp)
        elif t < n_st:
            issue(t, True)

    st = 0
    while st < n_final - rs:
        for r in range(rs):
            stage(st + r, True, False, False)
        st += rs
    if n_final >= rs:
        for r in range(rs):
            stage(n_final - rs + r, True, False, True)
    for r in range(rs):
        stage(n_final + r, r + 1 < rs, True, True)
    return sorted(issued), n_st


@pytest.mark.parametrize("k_stg", [2, 4])
@pytest.mark.parametrize("depth", [1, 2, 3])
@pytest.mark.parametrize("ring", [False, True])
def test_every_stage_once_and_unclamped_loads_in_the_data(k_stg, depth, ring):
    for nb in range(1, 800):
        issued, n_st = schedule(nb, k_stg, depth, ring)
        assert issued == list(range(n_st))


def test_unclamped_last_stage_is_caught():
    """The check itself: a ring-less tile that skipped the clamp in its main
    loop would issue the last stage unclamped."""
    def bad(nb, k_stg=4, depth=2):
        n_st = -(-nb // k_stg)
        for s in range(0, n_st - 2):
            t = s + 1 + depth
            if t < n_st and (t + 1) * k_stg > nb:
                return True
        return False
    assert any(bad(nb) for nb in range(1, 100))
