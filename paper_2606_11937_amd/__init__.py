"""TileChol: FP64 tiled right-looking Cholesky for MI355X (gfx950).

The compute path is the HIP library libtilechol.so behind the C ABI declared
in include/tilechol.h; `tilechol` is its thin ctypes binding.  The binding is
imported lazily so that the input recipes can be used without the library.
"""
__all__ = ["inputs", "tilechol"]
