"""Structure of the sweep kernel's gfx950 code that its memory waits rely on.

The sweep kernel stages rows into LDS with direct global-to-LDS loads and
waits for them with explicit ``s_waitcnt vmcnt(N)``: one counter covers
loads and stores and retires them in issue order, and every round issues its
9 N stores after its staging loads, so the next round waits until at most
9 N operations remain in flight.  That is exact only if

* every round's stores are exactly 9 N store instructions (none merged or
  split), and every explicit wait is vmcnt(0) or vmcnt(9 N);
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

KERNEL = re.compile(r"^(_ZN3lbm5sweep12k_sweep_d2q9INS_\d+(Store\w+?)ELi(\d)E\w*):", re.M)


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    if not shutil.which(B.HIPCC) and not os.path.exists(B.HIPCC):
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("isa") / "sweep.s"
    flags = [f for f in B.FLAGS if f not in ("-fPIC", "-Wall")]
    cmd = [B.HIPCC, *flags, "-S", "--cuda-device-only", os.path.join(B.CSRC, "k_sweep2d.hip"), "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True)
    return out.read_text()


def kernels(text):
    for m in KERNEL.finditer(text):
        end = text.index("s_endpgm", m.end())
        yield m.group(2), int(m.group(3)), text[m.end():end].split("\n")


def test_every_instantiation_present(asm):
    found = {(s, n) for s, n, _ in kernels(asm)}
    assert found == {(s, n) for s in ("StoreF32", "StoreF16S") for n in (1, 2, 3, 4)}


def test_stores_come_in_rounds_of_nine_n(asm):
    for store, nc, lines in kernels(asm):
        groups, cur = [], 0
        for line in lines:
            t = line.strip()
            if t.startswith(("global_store", "buffer_store", "flat_store")):
                cur += 1
            elif t.startswith(("global_", "buffer_", "flat_")) or ("s_waitcnt" in t and "vmcnt" in t):
                if cur:
                    groups.append(cur)
                cur = 0
        if cur:
            groups.append(cur)
        assert groups and all(g == 9 * nc for g in groups), (store, nc, groups)


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
                assert int(m.group(1)) in (0, 9 * nc), (store, nc, line.strip())


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
