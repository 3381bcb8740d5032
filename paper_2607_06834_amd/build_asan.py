"""Debug build of libptafs with the host code sanitized (CPU checks only).

build_host_asan() writes _build/asan/libptafs_asan.so: the host pass carries
AddressSanitizer and UndefinedBehaviorSanitizer, the device code is built as
in the product library.  It links the shared sanitizer runtime, so a process
that loads it preloads asan_runtime() first (LD_PRELOAD).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess

from .build import CSRC, FLAGS, HIPCC, INCLUDE, OUT_DIR, SOURCES  # noqa: F401

ASAN_DIR = os.path.join(OUT_DIR, "asan")
ASAN_LIB = os.path.join(ASAN_DIR, "libptafs_asan.so")
# host pass only: AddressSanitizer and UndefinedBehaviorSanitizer on the host
# code (descriptor checks, planning, G/QR and Gram precomputation, layouts);
# the device code is built as in the product library
ASAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]


def asan_runtime() -> str:
    """The compiler's shared ASan runtime, which a process must preload to
    load the sanitized library."""
    r = subprocess.run([os.path.join(os.path.dirname(HIPCC), "amdclang++"),
                        "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError(f"shared ASan runtime not found ({path or r.stderr.strip()})")
    return path


def _compile_asan(src):
    obj = os.path.join(ASAN_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *ASAN_HOST, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc (host ASan) failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build_host_asan() -> str:
    """Compile every source with the host pass sanitized and link them."""
    os.makedirs(ASAN_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile_asan, SOURCES))
    tmp = ASAN_LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-shared-libsan",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link (host ASan) failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, ASAN_LIB)
    return ASAN_LIB
