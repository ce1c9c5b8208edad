"""The paper's printed setup (tests/golden/paper_setup.json, Sec. IV-B, Sec.
III-B, Sec. IV-A) against the workloads and the readings built on it."""
import json
import os

import pytest

from paper_2301_08343_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_setup.json")


@pytest.fixture(scope="module")
def paper():
    with open(GOLDEN) as f:
        return json.load(f)


def test_printed_dataset_size_is_consistent(paper):
    """Sec. IV-A's count: positions x depths x indenters, depths 0..1 mm in
    0.1 mm steps."""
    lo, hi = paper["dataset_depth_range_mm"]
    depths = round((hi - lo) / paper["dataset_depth_step_mm"]) + 1
    assert depths == paper["dataset_images_per_position"]
    px, py = paper["dataset_positions"]
    assert px * py * depths * paper["dataset_indenters"] == paper["dataset_images"]


def test_gelsight_workload_has_the_paper_elastomer_and_image(paper):
    wl = W.gelsight_contact(seed=0, steps=10)
    cfg = wl["cfg"]
    assert [round(s * 1e3, 9) for s in cfg["block_size"]] == paper["elastomer_size_mm"]
    assert cfg["nu"] == paper["poisson_ratio"]
    assert [wl["render"]["h"], wl["render"]["w"]] == paper["image_hw"]
    # the configured modulus (0.15 MPa) is within 4 % of the printed one;
    # under a displacement-controlled press only the forces scale with it
    assert abs(cfg["E"] / paper["youngs_modulus_pa"] - 1) < 0.04


def test_paper_lattice_spacing_and_its_cell_centred_reading(paper):
    """R11: 101 particles over 20 mm (21 over 4 mm) is a vertex-centred
    lattice of 0.2 mm spacing; the cell-centred lattice at that spacing,
    the surrogate's data resolution, has 100 x 100 x 20 particles."""
    sizes, counts = paper["elastomer_size_mm"], paper["elastomer_particles"]
    spacing = [s / (n - 1) for s, n in zip(sizes, counts)]
    assert spacing == pytest.approx([0.2, 0.2, 0.2])
    wl = W.gelsight_contact_at(seed=0, h=spacing[0] * 1e-3, full=False)
    assert wl["cfg"]["n"] == (100, 100, 20)
    assert [round(s * 1e3, 9) for s in wl["cfg"]["block_size"]] == sizes


def test_paper_grid_is_finer_than_its_particles(paper):
    """Sec. IV-B prints a grid interval (33 mm over 256 nodes) below its
    particle spacing while stating that the grid interval should exceed the
    particle interval; the reading kept here is dx = h (one particle per
    cell), the stated principle at its limit, and the library rejects a grid
    finer than the lattice."""
    interval = paper["grid_edge_mm"] / paper["grid_nodes"][0]
    spacing = paper["elastomer_size_mm"][0] / (paper["elastomer_particles"][0] - 1)
    assert interval < spacing
    for cfg in (W.gelsight_contact(seed=1, steps=10)["cfg"], W.gelsight_contact_at(seed=1, full=False)["cfg"]):
        assert cfg["dx"] == pytest.approx(cfg["block_size"][0] / cfg["n"][0])
