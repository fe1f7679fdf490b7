"""CPU oracle (test infrastructure only; see set_oracle)."""
from .set_oracle import (LoopOracle, Oracle, VecLoopOracle, VecOracle, first_occurrence_flags,
                         first_occurrence_flags_vec, set_digest)

__all__ = ["LoopOracle", "Oracle", "VecLoopOracle", "VecOracle", "first_occurrence_flags",
           "first_occurrence_flags_vec", "set_digest"]
