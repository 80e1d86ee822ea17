"""CPU oracle for the gVOF path -- test infrastructure only (see oracle.py)."""
