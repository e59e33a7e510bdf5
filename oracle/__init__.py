"""TEST INFRASTRUCTURE ONLY: the CPU oracle (see oracle.py, pf_oracle.c)."""
