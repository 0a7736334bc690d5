"""MI355X-native G-prox PDHG solver for implicit reaction-diffusion steps.

The compute path is the HIP library ``librdpdhg.so`` (C ABI declared in
``include/rd.h``); ``paper_2305_03945_amd.rd`` is its thin ctypes binding.
Importing this package loads nothing; ``paper_2305_03945_amd.rd`` raises if the
built library is missing.  ``workloads`` holds the seeded synthetic inputs.
"""
