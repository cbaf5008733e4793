"""CPU oracle for the Torontonian (test infrastructure only; see oracle.py)."""
