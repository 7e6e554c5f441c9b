"""MI355X (gfx950) library for the Lattice Kinetic Scheme and its adjoint.

The compute path is the HIP library ``liblks.so`` (sources in ``csrc/``,
C ABI in ``include/lks.h``); ``lks`` is its ctypes binding and ``autograd``
wraps it in a torch.autograd.Function. ``workloads`` builds seeded
synthetic inputs. Submodules are imported on demand so that the input
generators can be used without the GPU library.
"""
