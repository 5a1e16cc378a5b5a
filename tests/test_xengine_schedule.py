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


def test_check_free_store_offsets():
    """The check-free epilogue stores of an interior off-diagonal 128-wide
    tile address baseline (a0 + k, b) as the lane's base plus k a0 + k (k+1)/2
    (a0 = i0 / 2 + 2 gb with gb in {0, 2}, k = 8 i + 2 h + r / 2 < 64, b below
    the tile's rows): the same baseline index as bl(a, b) = a (a + 1) / 2 + b,
    every baseline of the tile written exactly once per lane pair, and the
    byte offsets below 2^31 at the 4096-antenna limit."""
    def bl(a, b):
        return a * (a + 1) // 2 + b

    for Na in (576, 4096):
        N = 2 * Na
        n_side = -(-N // 128)
        max_off = 0
        for ti in range(n_side):
            i0 = ti * 128
            if i0 + 128 > N:
                continue                                    # edge tiles take the checked path
            for tj in (0, ti - 1) if ti > 0 else ():
                j0 = tj * 128
                seen = set()
                for gb in (0, 2):
                    a0 = i0 // 2 + 2 * gb
                    for col in range(128):                  # column receiver j0 + col, lane pair by antenna
                        b = (j0 + col) // 2
                        base = bl(a0, b)
                        for i in range(8):
                            for h in range(2):
                                for r in (0, 2):
                                    k = 8 * i + 2 * h + r // 2
                                    a = (i0 + 16 * i + 4 * (gb + h) + r) // 2
                                    assert a == a0 + k and a > b
                                    got = base + k * a0 + k * (k + 1) // 2
                                    assert got == bl(a, b)
                                    seen.add((a, b))
                                    max_off = max(max_off, got * 32 + 16)
                assert seen == {(a, b) for a in range(i0 // 2, i0 // 2 + 64) for b in range(j0 // 2, j0 // 2 + 64)}
        assert max_off < Na * (Na + 1) // 2 * 32 <= 2 ** 31
