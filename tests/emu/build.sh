#!/bin/bash
# Build libfr_emu.so in OUT (default $TMPDIR/fr_emu): the library's host code
# and its sparse-row, matrix-core and transformed-flux kernels compiled for
# the CPU with AddressSanitizer, every other kernel a no-op (stubs.cpp).
set -e
HERE="$(cd "$(dirname "$0")" && pwd)"
OUT="${1:-${TMPDIR:-/tmp}/fr_emu}"
mkdir -p "$OUT"
python3 "$HERE/gen.py" "$OUT"
FLAGS="-std=c++17 -O1 -g -fsanitize=address -fno-omit-frame-pointer -fPIC -I$HERE -I$OUT"
pids=()
for f in "$HERE/emu_rt.cpp" "$HERE/stubs.cpp" "$OUT/api.cpp" "$OUT/setup.cpp" "$OUT/gemm_host.cpp" "$OUT/emu_kernels.cpp"; do
  g++ $FLAGS -c "$f" -o "$OUT/$(basename "$f" .cpp).o" & pids+=($!)
done
for p in "${pids[@]}"; do wait "$p"; done
g++ -shared -fsanitize=address -o "$OUT/libfr_emu.so" "$OUT"/emu_rt.o "$OUT"/stubs.o "$OUT"/api.o \
    "$OUT"/setup.o "$OUT"/gemm_host.o "$OUT"/emu_kernels.o
echo "$OUT/libfr_emu.so"
