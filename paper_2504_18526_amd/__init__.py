"""SI-MLSDC with DG-SEM on MI355X: the HIP library ``libsisdc`` and its
Python binding.  See ``sisdc.py`` for the binding and ``include/sisdc.h``
for the C ABI."""
