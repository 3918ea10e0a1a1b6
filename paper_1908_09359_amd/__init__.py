"""MI355X (gfx950) hot path of variational Monte Carlo on finite open-boundary PEPS.

The compute path is the HIP library ``libvmcpeps.so`` behind the C ABI of
``include/vmcpeps.h``; ``binding`` is its ctypes wrapper and ``workloads``
holds the seeded synthetic inputs.  PyTorch is used only for device memory
and streams.
"""
