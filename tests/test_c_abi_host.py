"""The C ABI from C (no GPU): the public header compiles as strict C99 on its
own, and the C caller of the library compiles with the same flags."""
import os
import subprocess

from tests.c_abi import build_smoke

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_header_is_strict_c99(tmp_path):
    src = tmp_path / "h.c"
    src.write_text('#include "quadswarm.h"\n'
                   "int main(void) { qs_desc d; (void)d; return qs_error_string(QS_OK) == 0; }\n")
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-fsyntax-only",
                    "-I", os.path.join(ROOT, "include"), str(src)], check=True)


def test_c_caller_compiles():
    subprocess.run(["gcc", *build_smoke.c_flags(), "-fsyntax-only", build_smoke.SRC], check=True)
