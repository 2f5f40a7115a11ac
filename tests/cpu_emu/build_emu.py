"""CPU build of the library's HIP sources (a test tool for finding faults on the host).

The kernel sources are compiled unchanged for the host, except that every launch
`kernel<<<grid, block, shmem, stream>>>(args);` is rewritten into a call of the emulator's
synchronous launcher, and, with guard gaps on, every sub-buffer of the plan's workspace is
followed by a gap that the driver poisons for AddressSanitizer.  The result is a shared
library with the same C ABI as the GPU build (`libawe_emu.so`), whose device pointers are
host pointers.  Nothing in the product loads it.
"""
from __future__ import annotations

import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2304_05592_amd", "csrc")
SOURCES = ["awe_api.hip", "kernels2d.hip", "kernels3d.hip", "kernels_aux.hip", "schedule.cpp"]
CLANG = os.environ.get("EMU_CXX", "/opt/rocm/llvm/bin/clang++")
ASAN_RT = "/opt/rocm/llvm/lib/clang/{ver}/lib/linux/libclang_rt.asan-x86_64.so"
# bytes of poisoned gap after every workspace sub-buffer (EMU_GUARD widens it, so that an
# index that jumps whole fields past a sub-buffer's end still lands in a gap)
GUARD = int(os.environ.get("EMU_GUARD", "4096"))


def _kernel_start(text: str, i: int) -> int:
    """Start index of the kernel expression that ends right before text[i] ('<<<')."""
    j = i
    depth = 0
    while j > 0:
        c = text[j - 1]
        if c == ">":
            depth += 1
        elif c == "<":
            depth -= 1
        elif depth == 0 and not (c.isalnum() or c in "_:"):
            break
        j -= 1
    return j


def _balanced(text: str, i: int, open_c: str, close_c: str) -> int:
    """Index just past the bracket that closes text[i] (== open_c)."""
    depth = 0
    for j in range(i, len(text)):
        if text[j] == open_c:
            depth += 1
        elif text[j] == close_c:
            depth -= 1
            if depth == 0:
                return j + 1
    raise ValueError("unbalanced brackets")


def rewrite_launches(text: str) -> str:
    out = []
    pos = 0
    while True:
        i = text.find("<<<", pos)
        if i < 0:
            out.append(text[pos:])
            break
        k0 = _kernel_start(text, i)
        j = text.index(">>>", i)
        cfg = [c.strip() for c in _split_top(text[i + 3:j])]
        a0 = j + 3
        while text[a0].isspace():
            a0 += 1
        assert text[a0] == "(", text[k0:a0 + 20]
        a1 = _balanced(text, a0, "(", ")")
        kern = text[k0:i]
        args = text[a0 + 1:a1 - 1]
        out.append(text[pos:k0])
        out.append(f"::emu::launch(dim3({cfg[0]}), dim3({cfg[1]}), [&]() {{ {kern}({args}); }})")
        pos = a1
    return "".join(out)


def _split_top(s: str):
    """Split a launch configuration at top-level commas (not inside (), <> or [])."""
    parts, depth, cur = [], 0, ""
    for c in s:
        if c in "(<[":
            depth += 1
        elif c in ")>]":
            depth -= 1
        if c == "," and depth == 0:
            parts.append(cur)
            cur = ""
        else:
            cur += c
    parts.append(cur)
    return parts


GUARD_ALIGN_OLD = "long long align256(long long x) { return (x + 255) & ~255LL; }"

EMU_EXTRA = r'''
// ---- CPU build only: the workspace's sub-buffers, for the driver's guard gaps
extern "C" int awe_emu_subbuffers(const awe_plan* P, long long* out, int cap) {
  std::vector<long long> r;
  auto add = [&](long long off, long long n) { if (off >= 0 && n > 0) { r.push_back(off); r.push_back(off + n); } };
  add(0, (long long)awe::kReduceBlocks * 8);
  for (size_t w = 0; w < P->wins.size(); ++w) add(P->win_coef[w], P->wins[w].npts * 4);
  const int esz = P->store.prec == AWE_PREC_FP32 ? 4 : 2;
  for (const ShotDev& d : P->sd) {
    add(d.fld, (long long)awe::kFieldBufs * d.npts * 4);
    add(d.acc, d.npts * 8);
    if (P->store.mode == AWE_STORE_FULL) {
      add(d.store, (long long)d.nt * d.npts * esz);
      add(d.scale, (long long)d.nt * awe::kScaleSlots * 4);
    } else if (P->store.mode == AWE_STORE_CHECKPOINT) {
      add(d.store, (long long)P->store.nslots * 2 * d.npts * esz);
      add(d.scale, (long long)P->store.nslots * 2 * 4);
    } else if (P->store.mode == AWE_STORE_PROBED) {
      // the B and A probe sums as separate sub-buffers: an access of one past its end is caught
      add(d.store, (long long)P->store.nslots * d.npts * 8);
      add(d.store + (long long)P->store.nslots * d.npts * 8, (long long)P->store.nslots * d.npts * 8);
    }
  }
  const int n = (int)(r.size() / 2);
  for (int i = 0; i < n && i < cap; ++i) { out[2 * i] = r[2 * i]; out[2 * i + 1] = r[2 * i + 1]; }
  return n;
}
'''


def asan_runtime() -> str:
    base = "/opt/rocm/llvm/lib/clang"
    for ver in sorted(os.listdir(base)):
        p = ASAN_RT.format(ver=ver)
        if os.path.exists(p):
            return p
    raise FileNotFoundError("no clang AddressSanitizer runtime under " + base)


CKPT3D_GUARD = "store->mode == AWE_STORE_CHECKPOINT && prob->ndim == 3"


def build(out_dir: str = None, src_dir: str = CSRC, sanitize: bool = True, guard: bool = True,
          opt: str = "-O1", allow_3d_checkpoint: bool = True, include_dir: str = None,
          extra: str = None, verbose: bool = False) -> str:
    """Rewrite and compile the sources of src_dir into out_dir/libawe_emu.so; returns its path."""
    out_dir = out_dir or os.path.join(HERE, "_build")
    gen = os.path.join(out_dir, "src")
    os.makedirs(gen, exist_ok=True)
    for name in os.listdir(src_dir):
        if not name.endswith((".hip", ".h", ".cpp")):
            continue
        text = open(os.path.join(src_dir, name)).read()
        if name.endswith(".hip"):
            text = rewrite_launches(text)
        if name == "awe_api.hip" and guard:
            if GUARD_ALIGN_OLD not in text:
                raise RuntimeError("workspace alignment helper not found; update the guard rewrite")
            text = text.replace(GUARD_ALIGN_OLD,
                                f"long long align256(long long x) {{ return ((x + 255) & ~255LL) + {GUARD}; }}")
            text += EMU_EXTRA if extra is None else extra
        if name == "awe_api.hip" and allow_3d_checkpoint and CKPT3D_GUARD in text:
            text = text.replace(CKPT3D_GUARD, "false && " + CKPT3D_GUARD)
        dst = os.path.join(gen, name[:-4] + ".cpp" if name.endswith(".hip") else name)
        with open(dst, "w") as f:
            f.write(text)
    inc = ["-I", os.path.join(HERE, "shim"), "-I", include_dir or os.path.join(ROOT, "include"), "-I", gen]
    flags = ["-std=c++17", opt, "-g", "-fPIC", "-fno-omit-frame-pointer", "-Wno-unused-function",
             "-Wno-unused-variable"]
    if sanitize:
        flags += ["-fsanitize=address", "-shared-libasan"]
    objs = []
    srcs = [s[:-4] + ".cpp" if s.endswith(".hip") else s for s in SOURCES]
    for s in srcs + ["emu_runtime.cpp"]:
        path = os.path.join(HERE, s) if s == "emu_runtime.cpp" else os.path.join(gen, s)
        obj = os.path.join(out_dir, os.path.basename(s) + ".o")
        cmd = [CLANG] + flags + inc + ["-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    so = os.path.join(out_dir, "libawe_emu.so")
    subprocess.run([CLANG] + flags + ["-shared", "-o", so] + objs, check=True)
    return so


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
