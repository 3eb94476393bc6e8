"""The reference checker (test infrastructure only; see oracle.py)."""
