"""Plain FP64 CPU oracle of the GRPIC push + deposit step (test infrastructure only)."""
