"""Static check on the device assembly of the limb GEMM's epilogue.

The epilogue adds each output's triple share (and, for a continued K chunk,
the previous sum) and stores it.  Written per output as load-add-store, the
compiler cannot tell the output from the added terms and makes every load
wait for the store before it: a full `s_waitcnt vmcnt(0)` after each 8-byte
load, 16 memory round trips in a row per tile.  The kernels load every added
term before any store instead; this test compiles gemm_limb.hip for gfx950
with the library's own flags and checks that no 8-byte global load in the
kernels whose lanes own 16 outputs is followed at once by a full wait.  (No
GPU needed; skipped where hipcc is absent.)"""
import re

# kernels whose lanes own 16 outputs (every limb GEMM but the 128x64 and
# 64x128 tiles at one workgroup per compute unit, whose lanes own 32)
KERNELS = ("k_limb_gemmILi1ELi1E", "k_limb_gemm_ldsILi2ELi2E", "k_limb_gemm_ldsILi1ELi4E", "k_limb_gemm_ldsILi4ELi1E",
           "k_limb_gemm_sh", "k_limb_gemm_classes", "k_limb_gemm_persist")


def serial_loads(asm, names):
    """Per kernel: (8-byte global loads, those followed within two
    instructions by a full vector-memory wait)."""
    lines = asm.splitlines()
    out, fn = {}, None
    for i, line in enumerate(lines):
        m = re.match(r"^(_Z\S*):", line)
        if m:
            fn = m.group(1) if any(k in m.group(1) for k in names) else None
            if fn:
                out[fn] = [0, 0]
            continue
        if fn and re.search(r"\bglobal_load_dwordx2\b", line):
            out[fn][0] += 1
            if any("s_waitcnt" in x and "vmcnt(0)" in x for x in lines[i + 1:i + 3]):
                out[fn][1] += 1
    return out


def test_epilogue_loads_in_flight_together(limb_gemm_asm):
    st = serial_loads(limb_gemm_asm, KERNELS)
    # the direct 64x64 tile (schedule 2), six LDS-staged forms (schedules 5 to
    # 8, 12 and 13: the 64x64 tile, the three eight-wave tiles, the two thin
    # tiles), the three both-in-LDS forms (9 to 11), the classes kernel and
    # its persistent form
    assert len(st) == 12, sorted(st)
    for k, (loads, serial) in st.items():
        assert loads >= 32, (k, loads)  # the two groups of 16 added-term loads
        assert serial == 0, (k, loads, serial)


def test_parser_flags_serial_loads():
    asm = "\n".join([
        "_ZN3mpc12_GLOBAL__N_119k_limb_gemm_classesENS_10GemmTablesE:",
        "\tglobal_load_dwordx2 v[8:9], v[8:9], off",
        "\ts_waitcnt vmcnt(0)",
        "\tglobal_store_dwordx2 v[2:3], v[0:1], off",
        "\tglobal_load_dwordx2 v[10:11], v[10:11], off",
        "\tglobal_load_dwordx2 v[12:13], v[12:13], off",
        "\ts_waitcnt vmcnt(1)",
        "\ts_waitcnt vmcnt(0)",
    ])
    st = serial_loads(asm, KERNELS)
    assert list(st.values()) == [[3, 2]]
