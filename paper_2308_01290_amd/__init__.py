"""MI355X-native sinogram-domain one-step (Z, rho_e) estimation for dual-energy CT.

The compute path lives in the HIP library ``libdect.so`` (C-ABI, declared in
``include/dect.h``); :mod:`paper_2308_01290_amd.dect` is its thin ctypes
binding.  :mod:`paper_2308_01290_amd.phantoms` generates seeded synthetic inputs.
"""
