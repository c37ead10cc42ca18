"""Planted mistakes in a copy of the oracle must fail at least one pin.

Each case rewrites one line of sw_oracle.c the way a plausible bug would
(a wrong neighbour, a dropped factor, an off-by-one, a swapped word, ...),
builds the copy, routes the oracle module to it and runs the pins named
for that case; the test passes only if some pin rejects the mutant.
"""
import os

import pytest

import oracle
import test_oracle_pins as pins
import test_oracle_potts as potts
import test_oracle_cubic as cubic
import test_oracle_phi4 as phi4

SRC = os.path.join(os.path.dirname(oracle.__file__), "sw_oracle.c")
BETA_C = pins.BETA_C

MUTANTS = [
    ("bond uses <=", "&& wE < T) b |= 1u;", "&& wE <= T) b |= 1u;",
     [pins.test_bond_threshold_is_strict]),
    ("north neighbour is south", "return ((y + 1u) % L) * L + x;", "return ((y + L - 1u) % L) * L + x;",
     [lambda: pins.test_bond_keying_and_rule(6)]),
    ("bond word index", "uint32_t wN = r[2u * (s & 1u) + 1u];", "uint32_t wN = r[(s & 1u) + 1u];",
     [lambda: pins.test_bond_keying_and_rule(6)]),
    ("dropped factor 2 in p", "double p = -expm1(-2.0 * beta * J);", "double p = -expm1(-beta * J);",
     [pins.test_threshold_closed_form_at_beta_c, pins.test_4x4_exact_enumeration_chi2]),
    ("flip always word 0", "uint32_t bit = (r[(root >> 5) & 3u] >> (root & 31u)) & 1u;",
     "uint32_t bit = (r[0] >> (root & 31u)) & 1u;", [pins.test_assignment_uses_root_flip_bit]),
    ("labels keep the larger root", "if (ra < rb) parent[rb] = ra;", "if (ra > rb) parent[rb] = ra;",
     [lambda: pins.test_labels_equal_bfs(8)]),
    ("energy drops the N edges", "        e += si * spins[north_of(s, (uint32_t)L)];\n", "",
     [pins.test_records_and_invariants, pins.test_energy_at_beta_c_L64_matches_ferdinand_fisher]),
    ("cluster flips instead of being assigned", "spins[s] = (int8_t)orc_flip_spin(seed, t, labels[s]);",
     "spins[s] = (int8_t)(spins[s] * orc_flip_spin(seed, t, labels[s]));",
     [pins.test_spin_reversal_symmetry]),
    ("log2 bin off by one", "while ((sz >> (k + 1)) != 0u) ++k;", "while ((sz >> k) != 0u && k < 32) ++k;",
     [pins.test_records_and_invariants]),
    ("Philox multipliers swapped", "uint64_t prod_a = (uint64_t)0xD2511F53u * (uint64_t)x0;",
     "uint64_t prod_a = (uint64_t)0xCD9E8D57u * (uint64_t)x0;", [pins.test_philox_known_answers]),
    ("hot start inverted", "spins[s] = (r[0] & 1u) ? (int8_t)-1 : (int8_t)1;",
     "spins[s] = (r[0] & 1u) ? (int8_t)1 : (int8_t)-1;", [pins.test_init_hot_and_cold]),
    ("bond ignores the spins", "if (spins[s] == spins[east_of(s, (uint32_t)L)] && wE < T)", "if (wE < T)",
     [lambda: pins.test_bond_keying_and_rule(5), pins.test_4x4_exact_enumeration_chi2]),
    ("Potts p with the Ising factor 2", "double p = -expm1(-beta * J);", "double p = -expm1(-2.0 * beta * J);",
     [potts.test_threshold_closed_form, potts.test_q2_is_ising_at_half_the_coupling]),
    ("Potts value misses one state", "return (int8_t)(((uint64_t)w * q) >> 32);",
     "return (int8_t)(((uint64_t)w * (q - 1u)) >> 32);",
     [potts.test_init_and_value_ranges, potts.test_infinite_temperature_gives_iid_uniform_values]),
    ("Potts energy drops the N edges", "        e += spins[s] == spins[north_of(s, (uint32_t)L)];\n", "",
     [potts.test_infinite_temperature_gives_iid_uniform_values, potts.test_q3_critical_energy]),
    ("Potts cluster value from word 0", "return potts_value(r[root & 3u], (uint32_t)q);",
     "return potts_value(r[0], (uint32_t)q);", [potts.test_infinite_temperature_gives_iid_uniform_values]),
    ("cubic +z step goes to -z", "else z = (z + 1u) % L;", "else z = (z + L - 1u) % L;",
     [lambda: cubic.test_bond_keying_and_rule(0), lambda: cubic.test_labels_are_min_site_components(5, 0.25)]),
    ("cubic bond word of the next direction", "spins[s] == spins[nb] && r[d] < T",
     "spins[s] == spins[nb] && r[(d + 1) % 3] < T", [lambda: cubic.test_bond_keying_and_rule(3)]),
    ("cubic bonds on the 2D counter tag", "philox_seed(seed, s, t, 4u, r);", "philox_seed(seed, s, t, 0u, r);",
     [lambda: cubic.test_bond_keying_and_rule(0)]),
    ("cubic energy skips the +z edges", "for (int d = 0; d < 3; ++d) {\n            int8_t o",
     "for (int d = 0; d < 2; ++d) {\n            int8_t o",
     [cubic.test_2x2x2_ising_exact_enumeration_chi2, cubic.test_low_temperature_series]),
    ("cubic labels skip the +z bonds", "for (int d = 0; d < 3; ++d)\n            if (bonds[s] & (1u << d)) uf_union",
     "for (int d = 0; d < 2; ++d)\n            if (bonds[s] & (1u << d)) uf_union",
     [lambda: cubic.test_labels_are_min_site_components(4, 0.3), cubic.test_2x2x2_ising_exact_enumeration_chi2]),
    ("Potts hot start not random", "        spins[s] = potts_value(r[0], (uint32_t)q);",
     "        spins[s] = (int8_t)(s % (uint32_t)q);", [potts.test_hot_start_site_by_site_and_iid_uniform]),
    ("Potts hot start from word 1", "        spins[s] = potts_value(r[0], (uint32_t)q);",
     "        spins[s] = potts_value(r[1], (uint32_t)q);", [potts.test_hot_start_site_by_site_and_iid_uniform]),
    ("cubic Potts m_sum skips the last value",
     "for (int32_t k = 0; k < q; ++k)\n            if (count[k] > m) m = count[k];",
     "for (int32_t k = 0; k < q - 1; ++k)\n            if (count[k] > m) m = count[k];",
     [lambda: cubic.test_potts_m_sum_is_the_largest_population(3)]),
    ("phi4 bond with 2 kappa", "double k4 = 4.0 * kappa;", "double k4 = 2.0 * kappa;",
     [lambda: phi4.test_ring_energy_exact(8, 1.0), phi4.test_bond_rule_keying_and_probability]),
    ("phi4 projection not divided by r.r", "double a = ((px * py) * k4) / rr;", "double a = (px * py) * k4;",
     [lambda: phi4.test_ring_energy_exact(3, 0.3), phi4.test_bond_rule_keying_and_probability]),
    ("phi4 reflection without the factor 2", "double c = (2.0 * phi4_dot(f, r)) / rr;",
     "double c = phi4_dot(f, r) / rr;", [phi4.test_reflection_of_whole_clusters]),
    ("phi4 exp drops the last Taylor term", "for (int j = 13; j >= 1; --j) {", "for (int j = 13; j >= 2; --j) {",
     [phi4.test_expm_matches_library_exp]),
    ("phi4 reflection bit from word 0", "return (int32_t)((r[(root >> 5) & 3u] >> (root & 31u)) & 1u);",
     "return (int32_t)((r[0] >> (root & 31u)) & 1u);", [phi4.test_reflection_of_whole_clusters]),
    ("phi4 neighbour step goes backwards", "return x + 1u == L ? s - x * stride : s + stride;",
     "return x == 0u ? s + (L - 1u) * stride : s - stride;",
     [lambda: phi4.test_labels_are_min_site_components(4, 3), phi4.test_record_sums]),
    ("phi4 hot start not normalised", "for (int a = 0; a < 4; ++a) f[a] = v[a] / len;",
     "for (int a = 0; a < 4; ++a) f[a] = v[a];", [phi4.test_hot_and_cold_start]),
    ("phi4 bond keyed by the sweep of the direction", "philox_seed(seed, s, t, 7u, w);",
     "philox_seed(seed, s, t, 5u, w);", [phi4.test_bond_rule_keying_and_probability]),
]


@pytest.mark.parametrize("name,old,new,checks", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(name, old, new, checks, tmp_path):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not found once: {old!r}"
    so = oracle.build_variant(src.replace(old, new), str(tmp_path), "mutant")
    caught = []
    with oracle.using(so):
        for check in checks:
            try:
                check()
            except AssertionError:
                caught.append(check)
    assert caught, f"no pin caught the mutant '{name}'"
