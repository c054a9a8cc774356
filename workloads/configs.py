"""The workloads, as plain parameter dictionaries.

Units: length mm (or the scaled unit length for the unit-square case), time
ms, potential mV, capacitance per membrane area uF/mm^2, conductivity mS/mm,
current density per membrane area uA/mm^2.  ``stim_amp`` is I_stim (per
membrane area); a volumetric stimulus chi*I_stim = 50 uA/mm^3 therefore
becomes 50/chi.

Ionic models are named by the library's model enumeration: "HH" (classical
Hodgkin-Huxley), "LINEAR" (linear test model), "CRN_SURR" and "TTP_SURR"
(project-written surrogates with the variable counts and stiffness of the
Courtemanche-Ramirez-Nattel and ten Tusscher-Panfilov models).
"""
import copy

CHI_PHYS = 140.0     # 1/mm   (monodomain parameter table)
CM_PHYS = 0.01       # uF/mm^2

CONFIGS = {
    # unit square, 65x65 Q1 nodes, isotropic sigma=0.1, chi=Cm=1 (scaled units)
    "c1_2d_hh": dict(
        name="c1_2d_hh", kind="grid", dim=2, n=(65, 65), h=(1.0 / 64, 1.0 / 64),
        sigma=(0.1, 0.1, 0.1), chi=1.0, Cm=1.0, model="HH",
        stim=dict(kind="box", width=0.1, amp=20.0, t_on=0.0, t_off=1.0),
        dt=0.05, T=5.0, precision="fp64"),
    # 20 x 7 x 3 mm cuboid, h = 0.1 mm, fibres along x
    "c2_3d_crn": dict(
        name="c2_3d_crn", kind="grid", dim=3, n=(201, 71, 31), h=(0.1, 0.1, 0.1),
        sigma=(0.17, 0.019, 0.019), chi=CHI_PHYS, Cm=CM_PHYS, model="CRN_SURR",
        stim=dict(kind="box", width=1.5, amp=50.0 / CHI_PHYS, t_on=0.0, t_off=2.0),
        dt=0.05, T=50.0, precision="fp64"),
    # 60 x 60 x 10 mm slab, h = 0.1 mm, planar stimulus on the x = 0 face
    "c5_3d_crn_large": dict(
        name="c5_3d_crn_large", kind="grid", dim=3, n=(601, 601, 101), h=(0.1, 0.1, 0.1),
        sigma=(0.17, 0.019, 0.019), chi=CHI_PHYS, Cm=CM_PHYS, model="CRN_SURR",
        stim=dict(kind="face", axis=0, width=1.5, amp=50.0 / CHI_PHYS, t_on=0.0, t_off=2.0),
        dt=0.05, T=20.0, precision="fp64"),
}


def get_config(name, **overrides):
    cfg = copy.deepcopy(CONFIGS[name])
    cfg.update(overrides)
    return cfg


def small_config(base, n, **overrides):
    """Same physics as ``base`` on a smaller grid ``n`` (same spacing)."""
    cfg = get_config(base, **overrides)
    cfg["n"] = tuple(n)
    cfg["name"] = "%s_%s" % (base, "x".join(str(v) for v in n))
    return cfg


def stim_mask(cfg):
    from .grids import box_mask, face_mask
    st = cfg["stim"]
    if st["kind"] == "box":
        return box_mask(cfg["n"], cfg["h"][:cfg["dim"]], st["width"])
    if st["kind"] == "face":
        return face_mask(cfg["n"], cfg["h"][:cfg["dim"]], st["axis"], st["width"])
    if st["kind"] == "none":
        import numpy as np
        return np.zeros(int(__import__("numpy").prod(cfg["n"])), np.uint8)
    raise ValueError(st["kind"])
