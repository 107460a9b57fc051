"""FP64 CPU oracle of the upscaled Brinkman LBM.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.
"""
