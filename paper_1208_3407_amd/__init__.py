"""BITS (Binary Interval Search) on AMD Instinct MI355X (gfx950).

The compute path is the HIP library ``libbits.so`` behind the C ABI declared in
``include/bits.h``; ``paper_1208_3407_amd.bits`` is its thin Python binding
(argument marshalling only).  ``datagen`` samples the synthetic workloads.
"""
__all__ = ["bits", "datagen"]
