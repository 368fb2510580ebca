"""Plain FP64 CPU oracle of the elastoplastic hot path (test infrastructure only)."""
