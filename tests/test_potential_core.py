"""The potential-core helper on the host (no GPU): the region of Sec. 6
where the time-averaged axial velocity is at least 95 % of the inlet jet
velocity."""


def test_potential_core_mask():
    """Sec. 6: the potential core is where <U> >= 0.95 U_jet (host tensors;
    the helper only reads the mean axial velocity of stats_profiles)."""
    import torch
    from paper_2003_08746_amd import lesmi
    u_jet = 1.4
    y = torch.linspace(-2.0, 2.0, 41, dtype=torch.float64)[:, None]
    x = torch.arange(8, dtype=torch.float64)[None, :]
    # a core that narrows downstream: <U> = u_jet (1 - (|y| / (1 - x / 10))^2)
    half = 1.0 - x / 10.0
    u = u_jet * (1.0 - (y.abs() / half) ** 2)
    core = lesmi.potential_core({"u": u}, u_jet)
    expect = (y.abs() / half) ** 2 <= 0.05 + 1e-15
    assert core.dtype == torch.bool and core.shape == (41, 8)
    assert torch.equal(core, expect)
    # the core width shrinks monotonically downstream
    width = core.sum(0)
    assert (width[1:] <= width[:-1]).all() and width[0] > width[-1]
