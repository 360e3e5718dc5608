"""MI355X (gfx950) hot path of real-space parallel DMRG (Stoudenmire & White).

The computation lives in the HIP library ``libpdmrg.so`` (C ABI in
``include/pdmrg.h``); ``_lib`` is its ctypes binding and ``synth`` the seeded
synthetic-input generators.
"""
from . import synth            # noqa: F401
from ._lib import (F64, F32, BF16X3, SITE, TWO_SITE, ENV_L, ENV_R, ABSORB_RIGHT, ABSORB_LEFT,  # noqa: F401
                   SPLIT, Bond, Phys, MpoSite, Context, Heff, layout, lib, env_update,
                   davidson_step, merge_regions, PdmrgError)
