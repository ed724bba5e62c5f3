"""CPU oracle of the Viterbi decoder: test infrastructure only (see vref.h)."""
