"""Block-sparse matrix multiply with nonuniform block sizes on MI355X (gfx950).

``bsm``   -- ctypes binding of the C ABI in ``libbsm.so`` (include/bsm.h).
``gen``   -- seeded synthetic inputs.
``build`` -- compiles libbsm.so in-tree with hipcc.
Importing the package loads nothing; ``bsm.load()`` opens the library.
"""
