"""Bitsliced MICKEY 2.0 keystream generation on MI355X (gfx950).

The HIP kernels and the C-ABI live in ``csrc/`` and build into ``lib/libmickey.so``;
``mickey`` is the thin ctypes binding over that library (argument marshalling only).
``synth`` holds the seeded input recipes.
"""
__all__ = ["mickey", "synth"]
