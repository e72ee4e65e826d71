"""CPU oracle: test infrastructure only (see oracle/jagp.py)."""
