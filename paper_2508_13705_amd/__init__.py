"""MI355X-native ASE-DFF compact gas-kinetic scheme (arXiv 2508.13705).

The compute path is the HIP library ``libcgks.so`` (C ABI declared in
``include/cgks.h``); ``paper_2508_13705_amd.cgks`` is its thin ctypes binding.
``paper_2508_13705_amd.workloads`` builds seeded synthetic inputs.
"""
