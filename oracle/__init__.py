"""CPU oracle of IRT-PS: test infrastructure only (see oracle.py)."""
