"""Values the paper prints, kept as text fixtures under tests/golden/ with their citations:
the stated comparison configuration (section "Comparison of Deformation Results") against the
synthetic workload that stands in for it, and the composite encoding's width under the
encodings equation, read off the oracle."""
import os

import numpy as np

import nif_synth as S

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _fixture(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                key, value = line.split()
                vals[key] = int(value)
    return vals


def test_paper_workload_matches_the_stated_comparison_configuration():
    g = _fixture("paper_comparison_config.txt")
    w = S.workload("spheres32_paper")
    m = w.model
    assert w.N == g["voxel_resolution"]
    assert m.levels == g["hash_levels"]
    assert m.res[0] == g["hash_base_resolution"]
    assert m.feat_dim == g["hash_feature_dim"]
    assert m.pe_freqs == g["pe_bands"]


def test_oracle_encoding_width_of_the_comparison_configuration(orc):
    g = _fixture("paper_comparison_config.txt")
    m = S.workload("spheres32_paper").model
    rng = np.random.default_rng(7)
    tab = rng.normal(size=(m.levels, m.table_size, m.feat_dim))
    x = rng.uniform(0, 1, size=(16, 3))
    enc = orc.encode(m, tab, x)
    assert enc.shape == (16, g["encoding_width_per_point"])
    assert m.enc_width == 2 * g["encoding_width_per_point"]        # entry and exit points
