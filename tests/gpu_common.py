"""Helpers shared by the GPU tests: build the same problem for the HIP library and
for the FP64 oracle, run both, compare."""
import numpy as np


def rel_l2(a, b, mask):
    a = np.asarray(a, dtype=np.float64)[mask]
    b = np.asarray(b, dtype=np.float64)[mask]
    den = np.sqrt(np.sum(b * b))
    num = np.sqrt(np.sum((a - b) ** 2))
    return num / den if den > 0 else num


def make_gpu(rd, img, D, dx=1.0, robin=None, dirichlet=None, reactions=None, storage="fp32",
             B=8, sdf=None, features=0, checkpoint_slots=0, graph=True, xcd=True,
             kernel="block", wg_per_cu=8):
    g = rd.Geometry(img, sdf, dx, B)
    s = rd.Sim(g, storage)
    for d in D:
        s.add_species(d)
    for (a, b, k) in reactions or []:
        s.add_reaction(a, b, k)
    for sp, k in (robin or {}).items():
        s.set_robin(sp, k)
    for (sp, f), v in sorted((dirichlet or {}).items(), key=lambda kv: (kv[0][0], kv[0][1])):
        s.set_dirichlet(sp, f, v)
    s.set_launch(32, graph, xcd)
    s.set_kernel(kernel, wg_per_cu)
    s.bind(features=features, checkpoint_slots=checkpoint_slots)
    return g, s


def fields(s, n_species):
    import torch

    out = np.stack([s.get_field(i).cpu().numpy() for i in range(n_species)])
    torch.cuda.synchronize()
    return out.astype(np.float64)


def round_to_storage(x, storage):
    """The value a field holds after storing x in the given element type."""
    import torch

    t = torch.as_tensor(np.asarray(x, dtype=np.float32))
    if storage == "bf16":
        t = t.to(torch.bfloat16).to(torch.float32)
    elif storage == "fp16":
        t = t.to(torch.float16).to(torch.float32)
    return t.numpy().astype(np.float64)
