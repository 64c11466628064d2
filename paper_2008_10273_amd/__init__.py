"""MI355X-native block-based pseudodifferential residual decoding.

The compute path lives in the HIP/C-ABI library ``libpdinp.so`` (sources in
``csrc/``, header ``include/pdinp.h``); :mod:`paper_2008_10273_amd.binding`
marshals arguments to it.  :mod:`paper_2008_10273_amd.synth` draws seeded
synthetic inputs.  Importing this package loads nothing.
"""
__all__ = ["binding", "synth"]
