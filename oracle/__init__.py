"""FP64 CPU oracle of the sinogram-domain one-step (Z, rho_e) estimation.

TEST INFRASTRUCTURE ONLY.  Imported by tests/, by the smoke check and by the
CPU-baseline leg of the benchmark.  The product path (the HIP library and its
Python binding) never imports, links or calls anything in this folder, and this
folder imports nothing from the product package.
"""
