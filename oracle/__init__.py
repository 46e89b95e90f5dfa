"""FP64 CPU oracle (test infrastructure only; see ofm_oracle.py)."""
