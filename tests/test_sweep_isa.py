"""Structure of the sweep kernel's gfx950 code that its memory waits rely on.

The sweep kernel stages rows into LDS with direct global-to-LDS loads and
waits for them with explicit ``s_waitcnt vmcnt(N)``: one counter covers
loads and stores and retires them in issue order, and every round issues its
K stores after its staging loads (K = 9 N for FP32; 10 N for shifted FP16,
whose rows also store the sites' references), so the next round waits until
at most K operations remain in flight.  That is exact only if

* every round's stores are exactly K store instructions (none merged into a
  wider store or split), and every explicit wait is vmcnt(0) or vmcnt(K);
* the compiler adds no vmcnt wait of its own once staging has started (such
  a wait would also wait for the stores left in flight).

This test compiles the kernel source to gfx950 assembly with the library's
own flags and checks both, for every storage codec and component count the
kernel is built for.  It needs hipcc but no GPU.
"""
import os
import re
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_0704_3444_amd import build as B  # noqa: E402

KERNEL = re.compile(r"^(_ZN3lbm5sweep12k_sweep_d2q9INS_\d+(Store\w+?)ELi(\d)ELb(\d)E\w*):", re.M)


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    if not shutil.which(B.HIPCC) and not os.path.exists(B.HIPCC):
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("isa") / "sweep.s"
    flags = [f for f in B.FLAGS if f not in ("-fPIC", "-Wall")]
    cmd = [B.HIPCC, *flags, "-S", "--cuda-device-only", os.path.join(B.CSRC, "k_sweep2d.hip"), "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True)
    return out.read_text()


def kernels_w(text):
    for m in KERNEL.finditer(text):
        end = text.index("s_endpgm", m.end())
        yield m.group(2), int(m.group(3)), int(m.group(4)), text[m.end():end].split("\n")


def kernels(text):
    for s, n, _, lines in kernels_w(text):
        yield s, n, lines


def test_every_instantiation_present(asm):
    # periodic, and walls on y (separate instantiations); every structural
    # test below covers both
    found = sorted((s, n, w) for s, n, w, _ in kernels_w(asm))
    assert found == sorted((s, n, w) for s in ("StoreF32", "StoreF16S") for n in (1, 2, 3, 4) for w in (0, 1))


def stores_per_row(store, nc):
    return (10 if store == "StoreF16S" else 9) * nc


def blocks_of(lines):
    """Basic blocks of a kernel's assembly: (label, first, last) line ranges
    and the predecessors of each block."""
    label = re.compile(r"^(\.LBB\w+):")
    starts = [0]
    for i, l in enumerate(lines):
        t = l.strip()
        if label.match(t) and i not in starts:
            starts.append(i)
        elif t.startswith(("s_branch", "s_cbranch", "s_endpgm")) and i + 1 < len(lines):
            starts.append(i + 1)
    starts = sorted(set(starts))
    blocks = []
    for k, a in enumerate(starts):
        b = starts[k + 1] - 1 if k + 1 < len(starts) else len(lines) - 1
        m = label.match(lines[a].strip())
        blocks.append((m.group(1) if m else None, a, b))
    index = {lab: k for k, (lab, _, _) in enumerate(blocks) if lab}
    preds = [[] for _ in blocks]
    for k, (_, a, b) in enumerate(blocks):
        body = [lines[i].strip() for i in range(a, b + 1) if lines[i].strip() and not lines[i].strip().startswith(";")]
        last = body[-1] if body else ""
        if last.startswith(("s_branch", "s_cbranch")):
            target = last.split()[1]
            if target in index:
                preds[index[target]].append(k)
        if not last.startswith(("s_branch", "s_endpgm")) and k + 1 < len(blocks):
            preds[k + 1].append(k)
    return blocks, preds


def stores_since_last_load(lines, blocks, preds, at):
    """Numbers of store instructions on the paths from the nearest vector
    memory load back before line `at` to `at`, over every control path (a
    path that reaches an earlier vmcnt wait first stages nothing and is not
    counted)."""
    is_store = lambda t: t.startswith(("global_store", "buffer_store", "flat_store"))
    is_load = lambda t: t.startswith(("global_load", "buffer_load", "flat_load"))
    home = next(k for k, (_, a, b) in enumerate(blocks) if a <= at <= b)
    found, todo, seen = set(), [(home, at - 1, 0)], set()
    while todo:
        k, i, n = todo.pop()
        a = blocks[k][1]
        hit = False
        while i >= a:
            t = lines[i].strip()
            if is_load(t):
                found.add(n)
                hit = True
                break
            if "vmcnt" in t and "s_waitcnt" in t:
                # an earlier wait with no staging load after it: this path
                # stages nothing for the wait at `at` to protect
                hit = True
                break
            if is_store(t):
                n += 1
            i -= 1
        if hit:
            continue
        for q in preds[k]:
            if (q, n) not in seen:
                assert len(seen) < 100000, "a cycle without loads"
                seen.add((q, n))
                todo.append((q, blocks[q][2], n))
    return found


def test_stores_come_in_rounds_of_k(asm):
    """On every control path into an explicit vmcnt(K) wait, exactly K stores
    follow the last staging load (each slot its own store instruction: none
    merged, none split), so that the wait lets only those stores stay in
    flight; every store is a dword (FP32 slots, the rest slot) or a short
    (FP16 moving slots and references)."""
    checked = 0
    for store, nc, lines in kernels(asm):
        k = stores_per_row(store, nc)
        widths = {l.strip().split()[0] for l in lines
                  if l.strip().startswith(("global_store", "buffer_store", "flat_store"))}
        allowed = {"global_store_dword", "global_store_short"} if store == "StoreF16S" else {"global_store_dword"}
        assert widths and widths <= allowed, (store, nc, widths)
        blocks, preds = blocks_of(lines)
        for i, line in enumerate(lines):
            m = re.search(r"s_waitcnt\s.*vmcnt\((\d+)\)", line)
            if m and "ASMSTART" in lines[i - 1] and int(m.group(1)) == k:
                counts = stores_since_last_load(lines, blocks, preds, i)
                assert counts == {k}, (store, nc, i, counts)
                checked += 1
    assert checked > 0


def test_waits_after_staging_are_the_explicit_ones(asm):
    for store, nc, lines in kernels(asm):
        first_dma = min(i for i, l in enumerate(lines) if "global_load_lds" in l)
        for i, line in enumerate(lines):
            m = re.search(r"s_waitcnt\s.*vmcnt\((\d+)\)", line)
            if not m:
                continue
            explicit = "ASMSTART" in lines[i - 1]
            if i > first_dma:
                assert explicit, (store, nc, i, line.strip())
            if explicit:
                assert int(m.group(1)) in (0, stores_per_row(store, nc)), (store, nc, line.strip())


TILE_KERNEL = re.compile(r"^(_ZN3lbm12k_(fused|batch)_d2q9INS_\d+(Store\w+?)ELi(\d)E\w*):", re.M)


@pytest.fixture(scope="module")
def tile_asm(tmp_path_factory):
    if not shutil.which(B.HIPCC) and not os.path.exists(B.HIPCC):
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("isa") / "tile.s"
    flags = [f for f in B.FLAGS if f not in ("-fPIC", "-Wall")]
    cmd = [B.HIPCC, *flags, "-S", "--cuda-device-only", os.path.join(B.CSRC, "k_fused2d.hip"), "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True)
    return out.read_text()


def test_tile_kernels_use_global_memory_instructions(tile_asm):
    """The batched kernel reads its population pointers from the slot table;
    the tile step must still reach them with global (not flat) loads and
    stores, which would also count against the LDS counter."""
    kernels = 0
    for m in TILE_KERNEL.finditer(tile_asm):
        end = tile_asm.index("s_endpgm", m.end())
        body = tile_asm[m.end():end]
        kernels += 1
        assert "flat_load" not in body and "flat_store" not in body, m.group(1)
        assert "global_load" in body and "global_store" in body, m.group(1)
    assert kernels > 0


def test_tile_kernel_loads_are_not_serialised(tile_asm):
    """A component's pulled loads must be issued together: no global load is
    followed straight away by a wait for all loads (a branch and a wait
    around each 2-byte load once made the FP16 tile step twice as slow)."""
    for m in TILE_KERNEL.finditer(tile_asm):
        end = tile_asm.index("s_endpgm", m.end())
        lines = [l.strip() for l in tile_asm[m.end():end].split("\n")]
        serial = [j for j, l in enumerate(lines) if l.startswith("global_load")
                  and any(lines[j + d].startswith("s_waitcnt vmcnt(0)") for d in (1, 2) if j + d < len(lines))]
        assert len(serial) <= 8, (m.group(1), len(serial))


def test_sweep_kernels_inline_everything(asm):
    """The rounds' helpers must be inlined: a call passes their arrays through
    scratch memory, whose loads and stores are vector memory operations that
    the explicit vmcnt waits do not count."""
    for store, nc, lines in kernels(asm):
        body = "\n".join(lines)
        assert "s_swappc" not in body and "scratch_" not in body, (store, nc)


def test_shifted_fp16_decode_uses_mixed_precision_fmas(asm):
    """The shifted codec's decode (k_i h + d) and ledger (rest - d) are
    written so that they compile to v_fma_mix_f32, which converts its FP16
    operands itself; a factor the compiler could fold (1 or -1 as a
    constant) would turn them back into a conversion per operand plus an
    add.  Checked over each kernel: a handful of conversions at most."""
    for store, nc, lines in kernels(asm):
        if store != "StoreF16S":
            continue
        loop = [l.strip() for l in lines if l.strip() and not l.strip().startswith((";", "."))]
        mix = sum(1 for l in loop if l.startswith("v_fma_mix_f32"))
        cvt = sum(1 for l in loop if l.startswith("v_cvt_f32_f16"))
        # per row and component: 8 decoded moving slots, 8 ledger terms
        assert mix >= 16 * nc, (nc, mix, cvt)
        assert cvt <= 6 * nc, (nc, mix, cvt)  # 4 N today; 59 in the loop alone before


@pytest.fixture(scope="module")
def asm3d(tmp_path_factory):
    if not shutil.which(B.HIPCC) and not os.path.exists(B.HIPCC):
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("isa") / "sweep3d.s"
    flags = [f for f in B.FLAGS if f not in ("-fPIC", "-Wall")]
    cmd = [B.HIPCC, *flags, "-S", "--cuda-device-only", os.path.join(B.CSRC, "k_sweep3d.hip"), "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True)
    return out.read_text()


KERNEL3D = re.compile(r"^(_ZN3lbm6sweep313k_sweep_d3q19INS_\d+(Store\w+?)ELi(\d)ELb(\d)E\w*):", re.M)


def kernels3d(text):
    for m in KERNEL3D.finditer(text):
        end = text.index("s_endpgm", m.end())
        yield m.group(2), int(m.group(3)), int(m.group(4)), text[m.end():end].split("\n")


def m0_from_lane(lines):
    """Instructions that set M0 from a register written by v_readfirstlane."""
    from_lane, bad = set(), []
    for line in lines:
        t = line.strip().replace(",", " ").split()
        if not t:
            continue
        if t[0] == "v_readfirstlane_b32":
            from_lane.add(t[1])
        elif len(t) > 1 and t[1] == "m0":
            if set(t[2:]) & from_lane:
                bad.append(line.strip())
        elif len(t) > 1 and t[1] in from_lane:
            from_lane.discard(t[1])  # overwritten
    return bad


def test_d3q19_staging_destinations_are_uniform(asm3d):
    """The same check on the D3Q19 plane sweep's direct loads."""
    found = []
    for store, nc, walls, lines in kernels3d(asm3d):
        found.append((nc, walls))
        assert not m0_from_lane(lines), (store, nc, walls, m0_from_lane(lines))
    # N = 1 .. 3, periodic and walls on z
    assert sorted(found) == [(n, w) for n in (1, 2, 3) for w in (0, 1)]


def halo_unit_cover(lines, blocks, preds, at, n):
    """For the explicit vmcnt(n) at line `at`: over every control path back to
    the nearest direct 4-byte load into LDS (a halo-row unit load of the
    D3Q19 sweep), how many more vector memory operations that load would
    have needed after it to be complete at `at`.  Walking back, each vector
    memory operation lowers the need by one, and a wait vmcnt(m) on the way
    (the compiler's own, or an earlier explicit one) caps it at m, as that
    wait leaves only the m latest operations in flight.  A path whose value
    is above 0 would read the unit before it has landed."""
    is_unit = lambda t: t.startswith("buffer_load_dword ") and t.endswith(" lds")
    is_vmem = lambda t: t.startswith(("global_load", "buffer_load", "flat_load", "global_store", "buffer_store",
                                      "flat_store"))
    home = next(k for k, (_, a, b) in enumerate(blocks) if a <= at <= b)
    found, todo, seen = set(), [(home, at - 1, n)], set()
    while todo:
        k, i, need = todo.pop()
        a = blocks[k][1]
        hit = False
        while i >= a:
            t = lines[i].strip()
            if is_unit(t):
                found.add(need)
                hit = True
                break
            if is_vmem(t):
                need -= 1
            m = re.search(r"s_waitcnt\s.*vmcnt\((\d+)\)", t)
            if m:
                need = min(need, int(m.group(1)))
            i -= 1
        if hit:
            continue
        for q in preds[k]:
            if (q, need) not in seen:
                assert len(seen) < 100000, "a cycle without halo-row loads"
                seen.add((q, need))
                todo.append((q, blocks[q][2], need))
    return found


def test_d3q19_halo_unit_has_landed_at_its_wait(asm3d):
    """The D3Q19 sweep reads a plane's halo-row unit (direct loads into LDS,
    which the compiler does not track) after an explicit vmcnt(21): on every
    control path into that wait the unit's last load must be complete, by
    that wait (in the prologue the own unit's 19 loads and the 2 halo pieces
    of the next plane follow the unit, in the iterations those and the
    collision's 19 stores) or by the compiler's own waits for the own
    unit's register loads, issued after the unit and read just before.
    Checked for the periodic and the walled instantiations, whose wall
    planes take a branch of their own (there the compiler guards the second
    piece load with a branch on an empty lane mask, which the hardware never
    takes: lanes 0 .. 33 always load)."""
    checked = 0
    for store, nc, walls, lines in kernels3d(asm3d):
        blocks, preds = blocks_of(lines)
        for i, line in enumerate(lines):
            m = re.search(r"s_waitcnt\s.*vmcnt\((\d+)\)", line)
            if m and "ASMSTART" in lines[i - 1] and int(m.group(1)) == 21:
                needs = halo_unit_cover(lines, blocks, preds, i, 21)
                assert needs and max(needs) <= 0, (store, nc, walls, i, needs)
                checked += 1
    assert checked >= 6


def test_staging_destinations_are_uniform(asm):
    """A direct load's LDS destination is M0, one value for the whole wave.
    The compiler once merged a load issued by some lanes with the next load
    under divergent control flow and fed M0 from one lane of a per-lane
    choice of the two destinations (v_readfirstlane), so that the other
    lanes' data landed in the wrong place.  The staging loads are issued by
    the whole wave now; M0 must never come from a v_readfirstlane."""
    for store, nc, lines in kernels(asm):
        assert not m0_from_lane(lines), (store, nc, m0_from_lane(lines))
