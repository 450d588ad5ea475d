"""Regenerate philox_kat.txt from rocRAND's Philox4x32-10 engine, run on the host.

Each line: c0 c1 c2 c3 k0 k1 out0 out1 out2 out3 (decimal).  rocRAND is an
independent implementation of the published generator, so these vectors pin
both the oracle's and the GPU library's own Philox.
"""
import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))


def generate() -> str:
    with tempfile.TemporaryDirectory() as td:
        exe = os.path.join(td, "kat")
        subprocess.run(["hipcc", "-O1", "-x", "hip", "--offload-arch=gfx950", os.path.join(HERE, "rocrand_kat.cpp"),
                        "-o", exe], check=True)
        return subprocess.run([exe], check=True, capture_output=True, text=True).stdout


if __name__ == "__main__":
    txt = generate()
    with open(os.path.join(HERE, "philox_kat.txt"), "w") as f:
        f.write("# c0 c1 c2 c3 k0 k1 -> out0 out1 out2 out3 ; from rocRAND philox4x32_10 (host), "
                "written by make_philox_kat.py\n")
        f.write(txt)
    print(txt)
