"""Plain FP64 CPU oracle of the Yin-Yang AC direction-splitting step.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product package.
"""
