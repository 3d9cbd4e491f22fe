"""The public header is plain C99 and the library links into a C program.

Host only: the program calls the entry points that answer without a device
(version, workspace sizes, argument checks).
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_2208_07678_amd")

PROGRAM = r"""
#include "fec.h"
#include <stdio.h>

int main(void) {
    fec_server *srv = NULL;
    int64_t t = 0;
    printf("version %s\n", fec_version());
    printf("ws %d\n", fec_workspace_bytes(100000) > 0);
    printf("bws %d\n", fec_batch_workspace_bytes(100000, 8) > fec_workspace_bytes(100000));
    printf("einval %d\n", fec_cluster_async(NULL, 10, 0.0f, 1, 5, NULL, NULL, NULL, 0, NULL));
    printf("batch %d\n", fec_cluster_batch_async(NULL, 10, 0, NULL, NULL, NULL, NULL, NULL,
                                                 NULL, NULL, 0, NULL));
    printf("server %d\n", fec_server_create(1u << 30, 0, 8, &srv));
    printf("submit %d\n", fec_server_submit(NULL, NULL, 0, 0.3f, 1, 2, NULL, &t));
    printf("stages %d\n", fec_stage_count());
    printf("codes %d %d %d %d %d\n", FEC_OK, FEC_EINVAL, FEC_ERANGE, FEC_ENOMEM, FEC_EDEVICE);
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_header_is_c99_and_links(tmp_path):
    lib = os.path.join(LIBDIR, "libfec_hip.so")
    if not os.path.exists(lib):
        pytest.fail("HIP library not built: run python -m paper_2208_07678_amd.build")
    src = tmp_path / "prog.c"
    src.write_text(PROGRAM)
    exe = tmp_path / "prog"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic",
                    "-I", os.path.join(ROOT, "include"), str(src), "-L", LIBDIR,
                    "-l:libfec_hip.so", "-Wl,-rpath," + LIBDIR, "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    lines = dict(line.split(" ", 1) for line in out.strip().splitlines())
    assert lines["version"].startswith("fec-mi355x")
    assert lines["ws"] == "1" and lines["bws"] == "1"
    assert lines["einval"] == "-1" and lines["batch"] == "-1"
    assert lines["server"] == "-1" and lines["submit"] == "-1"
    assert int(lines["stages"]) > 10
    assert lines["codes"] == "0 -1 -2 -3 -4"
