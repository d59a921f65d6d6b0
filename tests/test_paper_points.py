"""Values the paper prints as plot coordinates (CPU): the points of its 3D diatomic convergence plot
(Section "Numerical Results"), read from the printed coordinates and the plot's logarithmic axis
ticks.  `tests/test_gpu_paper_experiments.py` compares the GPU path's errors with them."""
import json
import os


def paper_e5_points(golden_dir):
    """(grids N, step sizes, L2 density errors) of the 3D diatomic plot."""
    g = json.load(open(os.path.join(golden_dir, "paper_e5_points.json")))
    x0, x1 = g["x_ticks"]["1e-2"], g["x_ticks"]["1e-1"]
    y0, y1 = g["y_ticks"]["1e-4"], g["y_ticks"]["1e-2"]
    assert abs((g["y_ticks"]["1e-3"] - y0) - (y1 - g["y_ticks"]["1e-3"])) < 1e-3  # a log axis
    dts = [10.0 ** (-2.0 + (x - x0) / (x1 - x0)) for x, _ in g["points"]]
    errs = [10.0 ** (-4.0 + 2.0 * (y - y0) / (y1 - y0)) for _, y in g["points"]]
    return g["N"], dts, errs


def test_e5_points_sit_at_the_grids_of_table1(golden_dir):
    """The plot's x coordinates are the step sizes 2/N of Table 1's grids on [0, 2)^3, and the
    errors fall with the step size (about second order between the finer grids)."""
    Ns, dts, errs = paper_e5_points(golden_dir)
    assert Ns == [25, 40, 80, 120]
    for N, dt in zip(Ns, dts):
        assert abs(dt - 2.0 / N) < 2e-3 * dt, (N, dt)
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert 5e-3 < errs[0] < 7e-3 and 1.4e-4 < errs[-1] < 1.8e-4
