"""MI355X-native AIM (adaptive integral method) matvec, solve and RCS.

The compute path is the HIP library ``libaim.so`` (C ABI in include/aim.h);
``paper_1010_1456_amd.aim`` is its thin ctypes binding.
"""

from . import aim  # noqa: F401
from .aim import AIM_FP64, AIM_MIXED, Plan, host_plan, lib  # noqa: F401
