"""Static check on the device assembly of the LDS-staged limb GEMM.

Each k step of k_limb_gemm_lds (and of the classes kernels, one-shot and
persistent, that run its tile) hands its LDS buffers over at a barrier that
waits only until the wave's copies into LDS have landed: it lets the last
few vector-memory loads (the next step's inner planes, issued after the
copies) stay in flight.  Loads complete in issue order, so that wait is right
only if at least that many register loads follow the step's last copy in the
machine code.  The compiler's scheduling decides the final order, so this
test compiles the kernel for gfx950 with the library's own flags and checks
every hand-over.  (No GPU needed; skipped where hipcc is absent.)"""
import re


KERNELS = ("k_limb_gemm_lds", "k_limb_gemm_classes", "k_limb_gemm_persist")


def handovers(asm):
    """(kernel, waited vmcnt, register loads after the last LDS copy, LDS
    copies since the previous barrier) per barrier."""
    out, fn, seg, prev = [], None, [], ""
    for line in asm.splitlines():
        m = re.match(r"^(_Z\S*):", line)
        if m:
            fn = m.group(1) if any(k in m.group(1) for k in KERNELS) else None
            seg = []
        t = line.strip()
        if fn is None:
            prev = t
            continue
        if t.startswith("s_barrier"):
            w = re.search(r"vmcnt\((\d+)\)", prev)
            last_copy = max((i for i, x in enumerate(seg) if x == "copy"), default=-1)
            out.append((fn, int(w.group(1)) if w else None, sum(1 for x in seg[last_copy + 1:] if x == "load"),
                        seg.count("copy")))
            seg = []
        elif t.startswith("buffer_load") and t.endswith(" lds"):
            seg.append("copy")
        elif t.startswith(("buffer_load", "global_load")):
            seg.append("load")
        prev = t
    return out


def test_lds_handover_waits_cover_the_copies(limb_gemm_asm):
    hs = handovers(limb_gemm_asm)
    kernels = {h[0] for h in hs}
    # the eight LDS geometries (two of them thin), the classes kernel and its
    # persistent form
    assert len(kernels) == 10, kernels
    for k in kernels:
        assert sum(1 for h in hs if h[0] == k) >= 3, k  # prologue and steps
    for k, n, after, copies in hs:
        if copies == 0:
            continue  # hands over no LDS copy (the persistent kernel's tile-to-tile barrier)
        assert n is not None, (k, "barrier after LDS copies without a vmcnt wait before it")
        assert n == 0 or after >= n, (k, n, after)


def test_parser_flags_an_unsafe_wait():
    # synthetic machine code: the second step's copy comes after its loads
    asm = "\n".join([
        "_ZN3mpc12_GLOBAL__N_115k_limb_gemm_ldsILi1ELi2EEEvv:",
        "\tbuffer_load_dwordx4 v1, s[0:3], s4 offen lds",
        "\tbuffer_load_dwordx4 v[2:5], v6, s[0:3], s4 offen",
        "\tbuffer_load_dwordx4 v[6:9], v6, s[0:3], s4 offen",
        "\ts_waitcnt vmcnt(2) lgkmcnt(0)",
        "\ts_barrier",
        "\tbuffer_load_dwordx4 v[2:5], v6, s[0:3], s4 offen",
        "\tbuffer_load_dwordx4 v1, s[0:3], s4 offen lds",
        "\tbuffer_load_dwordx4 v[6:9], v6, s[0:3], s4 offen",
        "\ts_waitcnt vmcnt(2) lgkmcnt(0)",
        "\ts_barrier",
    ])
    hs = handovers(asm)
    assert [(n, after, copies) for _, n, after, copies in hs] == [(2, 2, 1), (2, 1, 1)]
    assert not all(n == 0 or after >= n for _, n, after, _ in hs)
