"""CPU oracle (test infrastructure only; see set_oracle)."""
from .set_oracle import LoopOracle, Oracle, first_occurrence_flags

__all__ = ["LoopOracle", "Oracle", "first_occurrence_flags"]
