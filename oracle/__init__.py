"""Plain FP64 CPU oracle of the Blacklight hot path -- test infrastructure only."""
