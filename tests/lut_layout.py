"""Views of a host image of the deferred-update tables, following the byte
layout the C header documents (test helper; the library itself is the
authority on the layout, and test_abi checks the sizes agree)."""
import numpy as np


def _al8(b):
    return (b + 7) // 8 * 8


def layout(T, K, nclass=0):
    nrow = (K if K > 0 else T) + 1
    o, L = 64, {"T": T, "K": K, "nrow": nrow}
    for name, size in (("Wf", 4 * 2 * nrow), ("Mf", 4 * nrow), ("Vf", 4 * nrow), ("SS", 4 * (T + 2)),
                       ("BC", 4 * (T + 2))):
        L[name] = o
        o += size
    o = _al8(o)
    for name, size in (("Wd", 8 * 2 * nrow), ("R", 8 * nrow), ("Cn", 8 * (T + 2))):
        L[name] = o
        o += size
    L["cls"] = o
    c = 0
    for name, size in (("Wlf", 4 * 2 * nrow), ("Pf", 4 * 2 * nrow), ("qf", 4 * (T + 2))):
        L["c" + name] = c
        c += size
    c = _al8(c)
    for name, size in (("Wld", 8 * 2 * nrow), ("Pd", 8 * 2 * nrow), ("qd", 8 * (T + 2))):
        L["c" + name] = c
        c += size
    L["cls_bytes"] = c
    L["total"] = o + nclass * c
    return L


def views(img, T, K, nclass=0):
    """dict of numpy views into the uint8 image `img`."""
    L = layout(T, K, nclass)
    n = L["nrow"]

    def f32(off, cnt, shape=None):
        a = img[off:off + 4 * cnt].view(np.float32)
        return a.reshape(shape) if shape else a

    def f64(off, cnt, shape=None):
        a = img[off:off + 8 * cnt].view(np.float64)
        return a.reshape(shape) if shape else a

    v = {"hdr": img[:64].view(np.int32), "Wf": f32(L["Wf"], 2 * n, (2, n)), "Mf": f32(L["Mf"], n),
         "Vf": f32(L["Vf"], n), "SS": f32(L["SS"], T + 2), "BC": f32(L["BC"], T + 2),
         "Wd": f64(L["Wd"], 2 * n, (2, n)), "R": f64(L["R"], n), "Cn": f64(L["Cn"], T + 2), "cls": []}
    for c in range(nclass):
        b = L["cls"] + c * L["cls_bytes"]
        v["cls"].append({"Wlf": f32(b + L["cWlf"], 2 * n, (2, n)), "Pf": f32(b + L["cPf"], 2 * n, (2, n)),
                         "qf": f32(b + L["cqf"], T + 2)})
    return v
