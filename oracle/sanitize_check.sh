#!/bin/sh
# Builds the C oracle with AddressSanitizer and UndefinedBehaviorSanitizer
# (gcc, host code only) and runs the oracle's pin tests against that build;
# any out-of-bounds access, use after free or undefined operation in
# sc_oracle.c aborts the run.  Test infrastructure, like the rest of oracle/.
set -e
HERE=$(cd "$(dirname "$0")" && pwd)
OUT=${TMPDIR:-/tmp}/sc_oracle_sanitized
mkdir -p "$OUT"
gcc -O1 -g -fno-omit-frame-pointer -fsanitize=address,undefined -fno-sanitize-recover=undefined \
    -std=gnu11 -fPIC -shared -pthread "$HERE/sc_oracle.c" -lm -o "$OUT/libsc_oracle.so"
RT="$(gcc -print-file-name=libasan.so) $(gcc -print-file-name=libubsan.so)"
cd "$HERE/.."
SC_ORACLE_LIB="$OUT/libsc_oracle.so" LD_PRELOAD="$RT${LD_PRELOAD:+ $LD_PRELOAD}" ASAN_OPTIONS=detect_leaks=0 \
    python -m pytest -q -x -m "not gpu" -p no:cacheprovider \
    tests/test_oracle_omp.py tests/test_oracle_sh.py tests/test_oracle_csc.py tests/test_oracle_dictlearn.py \
    tests/test_oracle_mlp.py tests/test_fixtures.py
