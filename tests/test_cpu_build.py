"""The library's HIP sources built for the CPU (tests/cpu_emu): kernels run as host code under
AddressSanitizer, with every gap between workspace sub-buffers poisoned, so an access that
leaves its own sub-buffer aborts the run with a report.  This is how the 3D checkpointed
gradient - refused on the GPU, see the design notes - is exercised: its launch sequence runs
clean, FP32 slots reproduce FULL storage bit for bit, and FP32 / BF16 slots match the oracle."""
import hashlib
import json
import os
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
EMU = os.path.join(HERE, "cpu_emu")
sys.path.insert(0, EMU)

pytestmark = pytest.mark.slow


def _sources_hash():
    import build_emu
    h = hashlib.sha256()
    for d in (build_emu.CSRC, os.path.join(EMU, "shim", "hip")):
        for name in sorted(os.listdir(d)):
            h.update(open(os.path.join(d, name), "rb").read())
    for name in ("emu_runtime.cpp", "build_emu.py"):
        h.update(open(os.path.join(EMU, name), "rb").read())
    return h.hexdigest()


@pytest.fixture(scope="module")
def emu_lib():
    """Build libawe_emu.so once per source state (about a minute)."""
    import build_emu
    out = os.path.join(EMU, "_build")
    stamp = os.path.join(out, "sources.sha256")
    so = os.path.join(out, "libawe_emu.so")
    key = _sources_hash()
    if not (os.path.exists(so) and os.path.exists(stamp) and open(stamp).read() == key):
        build_emu.build(out)
        with open(stamp, "w") as f:
            f.write(key)
    return so


def test_launch_rewrite_keeps_template_kernels_and_arguments():
    import build_emu
    src = "  case 4: k<TY, kStoreNone><<<a.ntiles, T3<TY>::NT, 0, s>>>(a, zlen(bz)); break;"
    out = build_emu.rewrite_launches(src)
    assert out == ("  case 4: ::emu::launch(dim3(a.ntiles), dim3(T3<TY>::NT), [&]() { k<TY, kStoreNone>"
                   "(a, zlen(bz)); }); break;")
    multi = "f<<<dim3(256, n, 2), kThreads, 0, s>>>(\n    a, slot);"
    assert "dim3(dim3(256, n, 2))" in build_emu.rewrite_launches(multi)


def test_3d_checkpointed_gradient_on_the_cpu_build(emu_lib):
    """FULL, CHECKPOINT FP32 and CHECKPOINT BF16 3D gradients on the CPU build, with the library's
    host-side launch checks on (every fill, slot copy and step range checked against the layout)."""
    import driver
    r = driver.run([os.path.join(EMU, "case_small.py")], emu_lib, {"CASE_T": "20", "CASE_CHECKS": "4"}, timeout=900)
    assert r.returncode == 0, r.stderr[-4000:]
    res = json.loads(r.stdout.strip().splitlines()[-1])
    print(res)
    assert res["poisoned_gaps"]
    assert res["fp32_slots_bitwise_full"]
    assert res["grad_rel_ckpt_fp32"] <= 1e-5 and res["traces_rel"] <= 1e-5
    assert 0 < res["grad_rel_ckpt_bf16"] <= 2e-2


def test_failure_paths_on_the_cpu_build(emu_lib):
    """AUTO storage falls back to CHECKPOINT under a mocked free-memory figure (bitwise the FULL
    gradient); input screening reports NaN (NONFINITE) and velocities above vmax (CFL) before any
    compute kernel; output screening reports a blow-up; the autotuner cache is written, and a
    cached entry is applied without running a kernel."""
    import driver
    r = driver.run([os.path.join(EMU, "case_failure_paths.py")], emu_lib, timeout=900)
    print(r.stdout[-2000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert r.stdout.strip().splitlines()[-1] == "CASE OK"


def test_two_level_tile_heights_on_the_cpu_build(emu_lib):
    """Two levels per launch at 8, 16, 24 and 32 rows (2D, uneven batch) under AddressSanitizer
    with the host launch checks on: bitwise the one-level gradient, traces and F^T dd (FULL FP32
    storage), which match the oracle, and bitwise the one-level Born traces."""
    import driver
    r = driver.run([os.path.join(EMU, "case_two_level.py")], emu_lib, timeout=900)
    assert r.returncode == 0, r.stderr[-4000:]
    res = json.loads(r.stdout.strip().splitlines()[-1])
    print(res)
    assert all(res["bitwise"].values()) and res["grad_rel"] <= 1e-5
    assert all(res["born_bitwise"].values())


def test_checkpointed_gradient_with_paired_two_level_reversals_on_the_cpu_build(emu_lib):
    """Checkpointed 2D gradients (uneven batch, 3 slots) whose paired reversals run two levels
    per launch, imaging from the recomputed forward levels, under AddressSanitizer with the host
    launch checks on: bitwise the FULL-storage one-level result with FP32 slots and the
    one-level result with BF16 slots, at 8, 16 and 24 rows and with one and two shot groups."""
    import driver
    r = driver.run([os.path.join(EMU, "case_ckpt_pairs.py")], emu_lib, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    res = json.loads(r.stdout.strip().splitlines()[-1])
    print(res)
    assert res["nonzero"] and all(res["bitwise"].values())

def test_probed_gradient_on_the_cpu_build(emu_lib):
    """PROBED storage on an uneven 2D batch against the oracle's gradient_probed (Rademacher
    probes) and against the exact gradient (identity table), and on a 3D shot (Rademacher), under
    AddressSanitizer; the result does not depend on the launch shape or the shot grouping."""
    import driver
    r = driver.run([os.path.join(EMU, "case_probed.py")], emu_lib, timeout=900)
    assert r.returncode == 0, r.stderr[-4000:]
    res = json.loads(r.stdout.strip().splitlines()[-1])
    print(res)
    assert res["rademacher"] <= 1e-5 and res["identity"] <= 1e-5 and res["identity_vs_exact"] <= 1e-5
    assert res["shape_invariant"]
    assert res["rademacher3d"] <= 1e-5 and res["shape_invariant3d"]
