"""FP64 CPU oracle for Time-Variant Overlap-Add in Partitions (TVOLAP).

TEST INFRASTRUCTURE ONLY. Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package. The GPU library and its
Python binding never import, call or link it; it shares no code with them.

Pins: every function here is checked in ``tests/test_oracle_pins.py`` against
results fixed by the paper or by mathematics independent of this code
(brute-force linear convolution, the time-domain block definition, a closed
form for IR switching, hand-worked examples, finite differences, an O(n^2)
DFT route with its own rounding for the reduced-precision form); the module
header of ``tvolap_ref`` names the pin of each function. ``comparators_ref``
(the comparison algorithms of Sec. 3) and ``nup_ref`` (non-uniform
partitions) are submodules with their own pins, named in their headers.
"""
from .tvolap_ref import *  # noqa: F401,F403
