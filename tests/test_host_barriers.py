"""The split-role barrier rule of the kernels whose wavefronts take different roles inside one
workgroup, checked on the sources (no GPU): a workgroup barrier inside a role-dependent branch is
correct only if every role meets the same number of barriers.

* F*Lambda (k_apply.hip): every role function (two reduced row blocks, one reduced and one FP64
  block, one FP64 block, the split contraction) runs the chunk loop fl_chunks exactly once and has
  no barrier of its own, except the split contraction, whose single extra barrier every wavefront
  of its (uniform) tile meets; the chunk loop itself has one barrier before its loop and one per
  chunk; the kernel body has no barrier and every branch of its role choice calls exactly one role
  function or the gather-only chunk loop.
* Pivoted Cholesky (k_krylov.hip): the factorising and the substituting wavefront each meet one
  set-up barrier and one barrier per step, and leave their step loops on the same stop mark.
* Deflation eigenproblem (k_deflation.hip): its only early exit precedes every barrier and depends
  on the subdomain alone (uniform over the workgroup)."""
import pathlib
import re

CSRC = pathlib.Path(__file__).resolve().parents[1] / "paper_2111_11728_amd" / "csrc"


def _body(src, signature_regex):
    m = re.search(signature_regex, src)
    assert m, signature_regex
    i = src.index("{", m.end() - 1)
    depth = 0
    for j in range(i, len(src)):
        if src[j] == "{":
            depth += 1
        elif src[j] == "}":
            depth -= 1
            if depth == 0:
                return src[i + 1:j]
    raise AssertionError("unbalanced braces")


def _strip_comments(src):
    src = re.sub(r"//[^\n]*", "", src)
    return re.sub(r"/\*.*?\*/", "", src, flags=re.S)


def test_flambda_roles_meet_the_same_barriers():
    src = _strip_comments((CSRC / "k_apply.hip").read_text())
    chunks = _body(src, r"__device__ __forceinline__ void fl_chunks\(")
    assert chunks.count("__syncthreads()") == 2
    assert re.search(r"store_x\([^;]*\);\s*__syncthreads\(\);\s*const int nch", chunks)   # before the loop
    loop = chunks[chunks.index("for (int ch = 0"):]
    assert loop.count("__syncthreads()") == 1 and "return" not in loop and "break" not in loop
    for fn in ("fl_fp32", "fl_bf16", "fl_fp64", "fl_mixed"):
        b = _body(src, r"__device__ __forceinline__ void " + fn + r"\(")
        calls = re.findall(r"\bfl_chunks(?:<[^>]*>)?\(", b)
        assert len(calls) == 1, fn
        assert "__syncthreads" not in b, fn
        assert "return" not in b.split(calls[0])[0], fn   # no exit before the chunk loop
    sk = _body(src, r"__device__ __forceinline__ void fl_fp64_splitk\(")
    assert sk.count("fl_chunks(") == 1 and sk.count("__syncthreads()") == 1
    assert sk.index("fl_chunks(") < sk.index("__syncthreads()")
    kern = _body(src, r"__global__ void __launch_bounds__\(kFLThreads\) k_flambda\(")
    assert "__syncthreads" not in kern
    # the tile-uniform exits come first; after them every branch makes exactly one call
    roles = kern[kern.index("const int nw_red"):]
    calls = re.findall(r"\b(fl_fp32|fl_bf16|fl_mixed|fl_fp64|fl_chunks)\s*<[^>]*>\s*\(|\b(fl_chunks)\s*\(", roles)
    names = [a or b for a, b in calls]
    assert sorted(names) == sorted(["fl_mixed", "fl_fp32", "fl_bf16", "fl_fp64", "fl_chunks"]), names
    # the mixed role returns right after its call; the reduced roles are the two arms of one
    # constexpr choice; the FP64 and gather-only roles are the other arms of the wave test
    assert re.search(r"fl_mixed<P, NB, Out>\([^;]*\);\s*return;", roles)
    assert re.search(r"if constexpr \(P == FETI_FP32\)\s*fl_fp32", roles)
    assert re.search(r"else if constexpr \(P == FETI_BF16X3\)\s*fl_bf16", roles)
    assert re.search(r"\}\s*else if \(wave >= nw_red[^{]*\{\s*fl_fp64<NB, Out>\([^;]*\);\s*\}\s*else \{\s*fl_chunks\(",
                     roles)
    head = kern[:kern.index("const int nw_red")]
    assert "fl_fp64_splitk<NB, Out>(" in head and re.search(r"if \(tl\.s < 0\) return;", head)


def test_pivchol_wavefronts_meet_the_same_barriers():
    src = _strip_comments((CSRC / "k_krylov.hip").read_text())
    kern = _body(src, r"__global__ void __launch_bounds__\(128\) k_pivchol\(")
    split = kern.index("if (w == 0) {")
    pre = kern[:split]
    assert pre.count("__syncthreads()") == 1        # the staged Gram matrix
    rest = kern[split:]
    # the factorising branch and the substituting branch
    i0 = rest.index("{")
    depth, j = 0, i0
    for j in range(i0, len(rest)):
        depth += rest[j] == "{"
        depth -= rest[j] == "}"
        if depth == 0:
            break
    fact, other = rest[i0 + 1:j], rest[j + 1:]
    assert other.lstrip().startswith("else")
    subst = _body(other, r"else \{")
    for branch in (fact, subst):
        loop = branch[branch.index("for (int m = 0") if "for (int m = 0" in branch else branch.index("for (; m < k"):]
        assert branch.count("__syncthreads()") == 2   # (S) and (B_m)
        assert loop.count("__syncthreads()") == 1
        assert "return" not in branch
    # both leave after the same barrier B_m on the same stop mark: the factorisation stops when no
    # pivot passes (p_s[m] = -1 is written before B_m), the substitution when it reads p_s[m] < 0
    assert re.search(r"if \(l == 0\) p_s\[m\] = p;\s*__syncthreads\(\);\s*if \(!go\) break;", fact)
    assert re.search(r"__syncthreads\(\);\s*const int p = p_s\[m\];\s*if \(p < 0\) break;", subst)


def test_deflation_eigenproblem_exit_is_uniform():
    src = _strip_comments((CSRC / "k_deflation.hip").read_text())
    kern = _body(src, r"__global__ void __launch_bounds__\(256\) k_defl_eig\(")
    first_barrier = kern.index("__syncthreads()")
    exits = [m.start() for m in re.finditer(r"\breturn\b", kern)]
    assert len(exits) == 1 and exits[0] < first_barrier
    cond = kern[:exits[0]]
    assert re.search(r"if \(n < 2 \* kP \|\| n > kDeflMaxNb\)", cond)   # n = the subdomain's n_b
