"""MI355X (gfx950) full-state quantum circuit simulator with profile-guided
gate fusion and virtual swaps (after QOPS, arXiv 2410.09326).

The simulation runs in libqops.so (hand-written HIP kernels); this package is
its ctypes binding.  There is no CPU fallback: importing the binding fails if
the library has not been built."""
from ._binding import (C64, C128, Batch, ORDER_LOGICAL, ORDER_PHYSICAL, PLAN_FUSED, PLAN_GATEWISE,  # noqa: F401
                       PLAN_LEARNED, PLAN_PROFILED, SWAP_PHYSICAL, SWAP_VIRTUAL, CostModel, GateArray, Plan, Profile, QopsError,
                       Simulator, TieredSimulator, lib, tier_plan)
