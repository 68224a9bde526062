"""FP64 CPU oracle of the decoupled pose search: test infrastructure, never on the product path."""
