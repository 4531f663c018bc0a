"""Pin for the setup-overlap model: every column of Table 4."""
import json
import os

import pytest

from oracle import setup_model as SM

TABLE = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table4_resnet50.json")))


@pytest.mark.parametrize("col", sorted(TABLE["columns"]))
def test_table4_column(col):
    s = TABLE["columns"][col]
    model = SM.serial_e2e if s["model"] == "serial" else SM.parallel_e2e
    assert model(s) == pytest.approx(s["e2e"], abs=0.05)


def test_serial_model_does_not_fit_parallel_columns():
    # the stage-3/4/cold columns are NOT sums: the overlap is real
    for col in ("stage3", "stage4", "cold"):
        s = TABLE["columns"][col]
        assert SM.serial_e2e(s) > s["e2e"] + 10
