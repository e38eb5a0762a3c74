"""FP64 CPU oracle (test infrastructure only; see oracle.py and rich_oracle.c)."""
