"""FP64 CPU oracle (test infrastructure only; see oracle/cwt.py)."""
