"""MI355X (gfx950) library for the coupled lattice-Boltzmann / dynamic
immersed-boundary step of Coclite, de Tullio, Pascazio and Politi (arXiv
2207.06043).  The compute path is the HIP library ``liblbmib.so`` behind the C
ABI in ``include/lbm.h``; this package only marshals arguments to it.
"""
from ._abi import (EXPORTS, LIB_PATH, LBM_E_DAMAGED, LBM_E_UNSTABLE, LBM_E_UNSUPPORTED, LBM_OK, Batch,
                   Lattice, LbmError, from_workload, load_library, trajectory)

from . import campaign  # noqa: E402

__all__ = ["campaign", "EXPORTS", "LIB_PATH", "LBM_E_DAMAGED", "LBM_E_UNSTABLE", "LBM_E_UNSUPPORTED", "LBM_OK", "Batch",
           "Lattice", "LbmError", "from_workload", "load_library", "trajectory"]
