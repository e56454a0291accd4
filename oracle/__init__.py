"""CPU oracle (test infrastructure only; see spinglass.py)."""
