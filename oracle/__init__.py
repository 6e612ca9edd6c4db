"""CPU oracle of the mechanical-interaction hot path: test infrastructure only (see oracle.py)."""
