"""Writes the instantiation tables of the fused sampling kernel.

Each table maps (dimension, map placement, training records) to one compiled
specialisation of k_sample; the specialisations are spread over several
translation units so that they compile in parallel.

    python paper_2009_05112_amd/csrc/gen_instances.py
"""
import os

HERE = os.path.dirname(os.path.abspath(__file__))

# file, function, precision, [(kind condition, kind constant, dims, helper, terms)], description
PRECS = [("fp64", "P_FP64", "double precision", "entry_for"),
         ("fp32acc", "P_FP32_ACC64", "single-precision map and integrand, double sums", "entry_for"),
         ("fp32neu", "P_FP32_NEUMAIER", "single-precision map and integrand, compensated single-precision sums",
          "entry_for_global_lds_only")]
TABLES = []
for tag, prec, desc, helper in PRECS:
    dmax = 16
    for kt in range(1, 5):
        TABLES.append((f"vp_sample_{tag}_gauss_k{kt}.hip",
                       f"sample_entry_{tag}_gauss_k{kt}(int dim, int map, bool rec)", prec,
                       [(None, "K_GAUSS_MIX", range(1, dmax + 1), helper, kt)],
                       f"{desc}, Gaussian mixture of {kt} term{'s' if kt > 1 else ''}, D = 1..{dmax}"))
TABLES += [
    ("vp_sample_fp64_corr.hip", "sample_entry_fp64_corr(int dim, int map, bool rec)", "P_FP64",
     [(None, "K_CORR_GAUSS", range(1, 25), "entry_for_global", 0)],
     "double precision, correlated-Gaussian integrand, D = 1..24"),
    ("vp_sample_fp64_generic.hip", "sample_entry_fp64_generic(int dim, int map, bool rec)", "P_FP64",
     [(None, "0", range(1, 25), "entry_for_global", 0)],
     "double precision, any integrand kind, D = 1..24"),
    ("vp_sample_fp64_batch.hip", "sample_entry_fp64_batch_acc(int dim, int map, bool rec)", "P_FP64",
     [(None, "K_BATCH_ACC", range(1, 25), "entry_for_global", 0)],
     "double precision, batched integrand (accumulation of the user's values), D = 1..24",
     ["SampleEntry sample_entry_fp64_batch_gen(int dim, int map)",
      "{",
      "    SampleEntry e = {nullptr, nullptr, 0};",
      "    switch (dim) {"] +
     [f"    case {d}: e = map == MAP_LDS ? make_entry<{d}, P_FP64, MAP_LDS, K_BATCH_GEN, false, 0>() "
      f": make_entry<{d}, P_FP64, MAP_GLOBAL, K_BATCH_GEN, false, 0>(); break;" for d in range(1, 25)] +
     ["    default: break;", "    }", "    return e;", "}", ""]),
    ("vp_sample_fp32acc_generic.hip", "sample_entry_fp32acc_generic(int dim, int map, bool rec)",
     "P_FP32_ACC64", [(None, "0", range(1, 17), "entry_for_global", 0)],
     "single-precision map and integrand, double sums, any integrand kind, D = 1..16"),
    ("vp_sample_fp32neu_generic.hip", "sample_entry_fp32neu_generic(int dim, int map, bool rec)",
     "P_FP32_NEUMAIER", [(None, "0", range(1, 17), "entry_for_global_lds_only", 0)],
     "single-precision map and integrand, compensated single-precision sums, any integrand kind, D = 1..16"),
    # mixed stratification (per-axis counts)
    ("vp_sample_fp64_generic_mix.hip", "sample_entry_fp64_generic_mix(int dim, int map, bool rec)", "P_FP64",
     [(None, "0", range(1, 25), "entry_for_global", "0, true")],
     "double precision, any integrand kind, mixed stratification, D = 1..24"),
    ("vp_sample_fp32acc_generic_mix.hip", "sample_entry_fp32acc_generic_mix(int dim, int map, bool rec)",
     "P_FP32_ACC64", [(None, "0", range(1, 17), "entry_for_global", "0, true")],
     "single-precision map and integrand, double sums, any integrand kind, mixed stratification, D = 1..16"),
    ("vp_sample_fp32neu_generic_mix.hip", "sample_entry_fp32neu_generic_mix(int dim, int map, bool rec)",
     "P_FP32_NEUMAIER", [(None, "0", range(1, 17), "entry_for_global_lds_only", "0, true")],
     "single-precision map and integrand, compensated single-precision sums, any integrand kind, "
     "mixed stratification, D = 1..16"),
    ("vp_sample_fp64_batch_mix.hip", "sample_entry_fp64_batch_acc_mix(int dim, int map, bool rec)", "P_FP64",
     [(None, "K_BATCH_ACC", range(1, 25), "entry_for_global", "0, true")],
     "double precision, batched integrand (accumulation of the user's values), mixed stratification, D = 1..24",
     ["SampleEntry sample_entry_fp64_batch_gen_mix(int dim, int map)",
      "{",
      "    SampleEntry e = {nullptr, nullptr, 0};",
      "    switch (dim) {"] +
     [f"    case {d}: e = map == MAP_LDS ? make_entry<{d}, P_FP64, MAP_LDS, K_BATCH_GEN, false, 0, true>() "
      f": make_entry<{d}, P_FP64, MAP_GLOBAL, K_BATCH_GEN, false, 0, true>(); break;"
      for d in range(1, 25)] +
     ["    default: break;", "    }", "    return e;", "}", ""]),
]


def switch(prec, kind, dims, helper, kt, indent):
    pad = " " * indent
    out = [f"{pad}switch (dim) {{"]
    for d in dims:
        out.append(f"{pad}case {d}: e = {helper}<{d}, {prec}, {kind}, {kt}>(map, rec); break;")
    out.append(f"{pad}default: break;")
    out.append(f"{pad}}}")
    return out


def render(fname, func, prec, parts, desc, extra=()):
    lines = [f"// {fname} -- instantiations of the fused sampling kernel: {desc}.",
             "// Written by gen_instances.py.",
             '#include "vp_sample.hpp"', "", "namespace vp {", ""]
    lines += list(extra)
    lines += [f"SampleEntry {func}", "{", "    SampleEntry e = {nullptr, nullptr, 0};"]
    for cond, kind, dims, helper, kt in parts:
        lines += switch(prec, kind, dims, helper, kt, 4)
    lines += ["    return e;", "}", "", "}  // namespace vp", ""]
    with open(os.path.join(HERE, fname), "w") as f:
        f.write("\n".join(lines))


def sources():
    """The generated translation units."""
    return [t[0] for t in TABLES]


def main():
    for t in TABLES:
        render(*t)


if __name__ == "__main__":
    main()
