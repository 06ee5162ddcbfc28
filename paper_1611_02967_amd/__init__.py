"""MI355X (gfx950) HIP solver for one time step of the second-order
convex-splitting scheme for Cahn-Hilliard-Hele-Shaw (arXiv 1611.02967).

The compute path is ``libchhs.so`` (HIP kernels behind the C ABI of
``include/chhs.h``); ``paper_1611_02967_amd.chhs`` is its ctypes binding and
``paper_1611_02967_amd.build`` compiles it.  Importing the binding without a
built library raises ImportError.
"""
