"""Identify a kernel of the built libmickey.so by its machine code.

A profile record (e.g. the rocprofv3 HBM-traffic summary of the headline kernel) is only
valid for the code it was measured on.  This module reads the gfx950 code objects that
hipcc embedded in the library (the `.hip_fatbin` section: clang offload bundles, one per
translation unit), finds the kernel's symbol and hashes its instruction bytes, so a record
stays valid across edits that do not change that kernel and lapses when the kernel does.
Only the library built from this repository is read.
"""
from __future__ import annotations

import hashlib
import struct

BUNDLE_MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"


def _sections(elf: bytes):
    """name -> (offset, size, addr) of an ELF64 little-endian image."""
    if elf[:4] != b"\x7fELF" or elf[4] != 2 or elf[5] != 1:
        raise ValueError("not an ELF64 little-endian image")
    shoff, = struct.unpack_from("<Q", elf, 0x28)
    shentsize, shnum, shstrndx = struct.unpack_from("<HHH", elf, 0x3A)
    hdrs = []
    for i in range(shnum):
        name, typ, flags, addr, off, size, link, info, align, entsize = struct.unpack_from(
            "<IIQQQQIIQQ", elf, shoff + i * shentsize)
        hdrs.append((name, typ, addr, off, size, link, entsize))
    stroff = hdrs[shstrndx][3]
    out = {}
    for k, (name, typ, addr, off, size, link, entsize) in enumerate(hdrs):
        end = elf.index(b"\0", stroff + name)
        out[elf[stroff + name:end].decode()] = (off, size, addr, k, link, entsize, typ)
    return out, hdrs


def _symbol_bytes(elf: bytes, symbol: str):
    secs, hdrs = _sections(elf)
    if ".symtab" not in secs:
        return None
    off, size, _, _, link, entsize, _ = secs[".symtab"]
    stroff = hdrs[link][3]
    for i in range(size // entsize):
        name, info, other, shndx, value, sz = struct.unpack_from("<IBBHQQ", elf, off + i * entsize)
        end = elf.index(b"\0", stroff + name)
        if elf[stroff + name:end].decode(errors="replace") == symbol and sz:
            s_addr, s_off = hdrs[shndx][2], hdrs[shndx][3]
            start = s_off + (value - s_addr)
            return elf[start:start + sz]
    return None


def device_code_objects(lib_path: str, target: str = "gfx950"):
    """Every device code object for `target` embedded in the library."""
    img = open(lib_path, "rb").read()
    secs, _ = _sections(img)
    off, size = secs[".hip_fatbin"][0], secs[".hip_fatbin"][1]
    fat = img[off:off + size]
    objs = []
    pos = fat.find(BUNDLE_MAGIC)
    while pos >= 0:
        n, = struct.unpack_from("<Q", fat, pos + len(BUNDLE_MAGIC))
        p = pos + len(BUNDLE_MAGIC) + 8
        for _ in range(n):
            e_off, e_size, t_size = struct.unpack_from("<QQQ", fat, p)
            triple = fat[p + 24:p + 24 + t_size].decode()
            p += 24 + t_size
            if triple.endswith(target) and e_size:
                objs.append(fat[pos + e_off:pos + e_off + e_size])
        pos = fat.find(BUNDLE_MAGIC, pos + 1)
    return objs


def kernel_code_hash(lib_path: str, symbol: str) -> str | None:
    """sha256 (16 hex digits) of the kernel's instruction bytes, or None if not found."""
    for co in device_code_objects(lib_path):
        code = _symbol_bytes(co, symbol)
        if code is not None:
            return hashlib.sha256(code).hexdigest()[:16]
    return None
