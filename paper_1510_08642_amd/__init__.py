"""MI355X-native double-double / quad-double matrix products and DD LU.

The compute path is the HIP library ``libddqd.so`` (built for gfx950) behind
a C ABI; :mod:`paper_1510_08642_amd.ddqd` is its thin ctypes binding over
torch device tensors.  :mod:`paper_1510_08642_amd.inputs` holds the seeded
input generators.
"""
