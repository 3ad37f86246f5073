"""GMT* (Group Marching Tree) hot path for AMD Instinct MI355X (gfx950).

Submodules are imported explicitly so that importing the package costs nothing:

* ``paper_1705_02403_amd.gmt``    -- ctypes binding of ``libgmt.so`` (the C ABI in
  ``include/gmt.h``); every planning step runs in the library's HIP kernels.
* ``paper_1705_02403_amd.inputs`` -- seeded synthetic problems (box worlds, sample
  sets, start states, goal balls); it holds no planning arithmetic.
* ``paper_1705_02403_amd.radius`` -- the connection radius of Theorem 1.
"""

__all__ = ["gmt", "inputs", "radius"]
