"""Oracle: plain, slow, obviously correct CPU references (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, the package smoke check and the benchmark's CPU-baseline leg may
import anything here. The product path never does; it shares no code with this
package and fails loudly when its HIP library is missing.

* ``sw2d_ref``  - FP64 C loops for the 2DSW step and its per-step folds.
* ``exact``     - the same step in exact rational arithmetic (tiny grids).
"""
