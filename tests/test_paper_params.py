"""The synthetic workloads take the paper's printed parameters where the
paper gives them (Tables S2-S3): seed, initial T_eff, activation parameters,
hit distance."""
import json
import os

from paper_2609_31258_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_params.json")


def test_configs_use_paper_parameters():
    P = json.load(open(GOLDEN))
    s2, rb = P["table_s2"], P["table_s3"]["rhodamine_b"]
    assert synth.SEED == s2["random_seed"]
    for cfg in (synth.config_c1, synth.config_c1t, synth.config_c2):
        f, ions, srcs, op, _ = cfg()
        assert op.d_hit == s2["electrode_hit_distance_m"]
        for ion in ions:
            assert ion.t_eff0 == rb["t_eff0_k"]
            assert (ion.act_kind, ion.act_p1, ion.act_p2) == (1, rb["dH_j_per_mol"], rb["dS_j_per_mol_k"])
    for ion in synth.config_c5_species():
        assert ion.t_eff0 == rb["t_eff0_k"] and ion.act_kind == 2 and ion.act_p1 == 1e12
