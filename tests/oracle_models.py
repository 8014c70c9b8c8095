"""Oracle model builders shared by the tests (test-side helper)."""
import oracle as O
from paper_2404_07780_amd import synth as S


def from_spec(name: str, oversample: int = 10, os_window: int = 5) -> O.Model:
    spec = S.MODEL_SPECS[name]
    return O.Model([O.Comp(t, bool(c), idx, fx) for t, c, idx, fx in spec["comps"]], spec["p"],
                   oversample=oversample, os_window=os_window)


def single(type_: int, convolve: bool = True, fixed=None, sky: bool = False, oversample: int = 10,
           free=None, box: bool = False, shape: bool = False) -> O.Model:
    """One component with every slot free (except shape constants -- Ferrer a,
    b and King alpha are free with `shape` -- and the Sersic boxiness unless
    `box`), plus an optional sky column at the end."""
    slots = O.SLOTS[type_]
    idx, fx, k = [], [], 0
    for s, name in enumerate(slots):
        if ((name in ("a", "b", "alpha") and not shape) or name == "beta" or (name == "box" and not box)
                or (free is not None and name not in free)):
            idx.append(-1)
            fx.append((fixed or {}).get(name, 0.0))
        else:
            idx.append(k)
            fx.append(0.0)
            k += 1
    comps = [O.Comp(type_, convolve, idx, fx)]
    if sky:
        comps.append(O.Comp(O.SKY, False, [k], []))
        k += 1
    return O.Model(comps, k, oversample=oversample)


def to_gm(model: O.Model):
    """The same model description for the HIP library's binding."""
    from paper_2404_07780_amd import gmfit as G

    return G.Model([G.Component(c.type, c.convolve, list(c.idx), list(c.fixed)) for c in model.comps], model.p,
                   m0=model.m0, oversample=model.oversample, os_window=model.os_window)
