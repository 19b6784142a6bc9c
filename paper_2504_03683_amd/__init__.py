"""MI355X-native exact trace tally (THAPI-style Tally/Interval analysis on gfx950).

The compute path is the HIP library libthapi_tally.so behind the C ABI of
include/thapi_tally.h; this package only binds it (tally.py), builds it
(build.py) and formats results (report.py).
"""
from .tally import (ALL, DEVICE_INPUT, DROP_ON_FULL, FMT_FIXED24, FMT_VAR16, NONBLOCKING, PROFILE,
                    SCOPE_FN, SCOPE_KERNEL, SCOPE_PROCESS, SCOPE_THREAD, STRICT, Tally, TallyError)

__all__ = ["Tally", "TallyError", "FMT_FIXED24", "FMT_VAR16", "DEVICE_INPUT", "NONBLOCKING", "DROP_ON_FULL",
           "STRICT", "PROFILE", "SCOPE_THREAD", "SCOPE_PROCESS", "SCOPE_FN", "SCOPE_KERNEL", "ALL"]
