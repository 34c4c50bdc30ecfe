"""Plant mistakes in the oracle (on the CPU) and check that its pins catch each one.

Every mutant is a build of oracle.c with one preprocessor switch that introduces
a plausible bug; at least one pin must fail on it."""
import os

import pytest

import oracle
from tests import pins_oracle

MUTANTS = {
    "ORACLE_MUTANT_SHORT_COPY": [pins_oracle.pin_retrieve_brute_force],
    "ORACLE_MUTANT_NEIGHBOUR": [pins_oracle.pin_retrieve_brute_force, pins_oracle.pin_retrieve_closed_forms],
    "ORACLE_MUTANT_TIES_DESCENDING": [pins_oracle.pin_sort_ties],
    "ORACLE_MUTANT_UNSTABLE_JOIN": [pins_oracle.pin_join_dim_order],
    "ORACLE_MUTANT_HASH_LAST": [pins_oracle.pin_hash_build_invariants],
    "ORACLE_MUTANT_LOOKUP_LAST": [pins_oracle.pin_hash_lookup_brute_force],
    "ORACLE_MUTANT_SMJ_J_MAJOR": [pins_oracle.pin_smj_brute_force, pins_oracle.pin_smj_closed_forms],
    "ORACLE_MUTANT_BTREE_FIRST_ENTRY": [pins_oracle.pin_btree_structure, pins_oracle.pin_btree_lookup_brute_force],
    "ORACLE_MUTANT_BTREE_STRICT": [pins_oracle.pin_btree_lookup_brute_force],
    "ORACLE_MUTANT_KEYJOIN_LAST_MATCH": [pins_oracle.pin_key_join_brute_force],
}


@pytest.mark.parametrize("define", sorted(MUTANTS))
def test_pins_catch_mutant(define, tmp_path):
    path = oracle.build(defines=(define,), out_path=os.path.join(tmp_path, f"lib_{define}.so"))
    lib = oracle.load(path)
    for pin in MUTANTS[define]:
        with pytest.raises(AssertionError):
            pin(lib)
