"""MI355X-native solver for the inviscid variable-density artificial-compressibility equations
with dual time stepping (Leakey, Glenis & Hewett, arXiv:2108.08769).

The solver is the HIP library ``libvdac.so`` behind the C ABI of ``include/vdac.h``;
``paper_2108_08769_amd.vdac`` is its thin Python binding and ``workloads`` builds the seeded
synthetic inputs.  Build with ``python -m paper_2108_08769_amd.build``.
"""
__all__ = ["vdac", "workloads", "build"]
