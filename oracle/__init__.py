"""Plain FP64 CPU oracle (test infrastructure only).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg use this
package.  The product library never imports it.
"""
from .oracle import *  # noqa: F401,F403
