"""Host-compilable copies of the library's sources for the emulation in this
directory: kernel launches become calls of emu_launch (every thread of the
grid in turn), and the matrix-core instructions become no-ops on the
accumulator (no address depends on their values).

    python3 tests/emu/gen.py OUTDIR
"""
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(ROOT, "paper_1312_1638_amd", "csrc")


def rewrite_launches(text):
    # K<...><<<grid, block, shmem, stream>>>(args);  ->  emu_launch(grid, block, [=]() { K<...>(args); });
    pat = re.compile(r'(\b\w+<[^;{}]*?>)<<<\s*([^,>]+)\s*,\s*(\d+)\s*,\s*[^,>]+,\s*\w+\s*>>>\s*\((.*?)\);',
                     re.S)
    return pat.sub(lambda m: f"emu_launch({m.group(2)}, {m.group(3)}, [=]() {{ {m.group(1)}({m.group(4)}); }});",
                   text)


def body(path):
    """The contents of a file's `namespace fr { ... }` block."""
    t = open(path).read()
    i = t.index("namespace fr {\n") + len("namespace fr {\n")
    j = t.rindex("}  // namespace fr")
    return t[i:j]


def main(out):
    os.makedirs(out, exist_ok=True)
    for f in ["spop.h", "kernels.h", "physics.h", "buffer.h", "setup.h", "adjoint.h", "steppers.h",
              "gemm.h"]:
        t = rewrite_launches(open(os.path.join(SRC, f)).read())
        if f == "gemm.h":
            t = t.replace("typedef double dbl4 __attribute__((ext_vector_type(4)));",
                          "typedef double dbl4 __attribute__((vector_size(32)));")
            t = t.replace("typedef float flt4 __attribute__((ext_vector_type(4)));",
                          "typedef float flt4 __attribute__((vector_size(16)));")
            t = t.replace("__builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0)", "((void)a, (void)b, c)")
            t = t.replace("__builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0)", "((void)a, (void)b, c)")
        assert "<<<" not in t, f
        open(os.path.join(out, f), "w").write(t)
    # the transformed-flux kernel and its launchers
    k = open(os.path.join(SRC, "kernels.hip")).read()
    kern = k[k.index("template <int D, int NS, typename TQ, bool MULTI = false>"):
             k.index("static inline unsigned blocks_for")]
    launch = k[k.index("template <typename TQ, bool MULTI>\nstatic hipError_t tflux_m"):
               k.index("hipError_t launch_devstate")]
    c = k.index("hipError_t launch_tflux(const PointArgs &a, int ns, hipStream_t s) {")
    d = k.index("}\n", c) + 2
    kernels = ['#include "spop.h"', '#include "gemm.h"', "namespace fr {",
               body(os.path.join(SRC, "spop.hip")), body(os.path.join(SRC, "spop_fields.hip")),
               body(os.path.join(SRC, "gemm_f64.hip")), body(os.path.join(SRC, "gemm_f32.hip")),
               "hipError_t launch_spop_lds_f64(int, const GemmArgs &, const StagedOp &, int, hipStream_t)"
               " { return hipSuccess; }",
               "hipError_t launch_spop_lds_f32(int, const GemmArgs &, const StagedOp &, int, hipStream_t)"
               " { return hipSuccess; }",
               kern, "static inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }",
               rewrite_launches(launch), k[c:d], "}  // namespace fr"]
    t = "\n".join(kernels)
    assert "<<<" not in t
    open(os.path.join(out, "emu_kernels.cpp"), "w").write(t)
    api = open(os.path.join(SRC, "api.cpp")).read()
    api = api.replace('#include "../../include/fr.h"', '#include "' + os.path.join(ROOT, "include", "fr.h") + '"')
    open(os.path.join(out, "api.cpp"), "w").write(api)
    for f in ["setup.cpp", "gemm_host.cpp"]:
        open(os.path.join(out, f), "w").write(open(os.path.join(SRC, f)).read())


if __name__ == "__main__":
    main(sys.argv[1])
