#!/bin/bash
# build_sanitized.sh SANITIZER OUTDIR -- the library's sources and the C ABI driver
# (tests/native/abi_sanitized.cpp) built into one executable, OUTDIR/abi_SANITIZER, with
# the host code instrumented by SANITIZER (address; thread builds too, but the ROCm runtime
# finds no device under ThreadSanitizer's memory layout).  The gfx950 device code is
# compiled as in the library build; the sanitizer applies to host code only, so every
# -fsanitize below follows -Xarch_host on the hipcc lines, and the host-only sources go
# through clang++ (one runtime for the whole program).
set -euo pipefail
SAN=$1
OUT=$2
ROOT=$(cd "$(dirname "$0")/../.." && pwd)
CSRC=$ROOT/paper_1609_08146_amd/csrc
HIPCC=/opt/rocm/bin/hipcc
CLANG=/opt/rocm/llvm/bin/clang++
mkdir -p "$OUT"
FLAGS="--offload-arch=gfx950 -O2 -g -std=c++17 -fPIC -ffp-contract=off -Xclang -target-feature -Xclang -packed-fp32-ops -Wno-unused-result -Wno-pass-failed -I $ROOT/include"
pids=()
for s in sc_quad.hip sc_kernels.hip sc_diag.hip; do
    $HIPCC $FLAGS -Xarch_host -fsanitize=$SAN -Xarch_host -fno-omit-frame-pointer -c "$CSRC/$s" -o "$OUT/${s%.hip}.o" &
    pids+=($!)
done
for s in sc_api.cpp sc_serve.cpp; do
    $HIPCC -x hip $FLAGS -Xarch_host -fsanitize=$SAN -Xarch_host -fno-omit-frame-pointer -c "$CSRC/$s" -o "$OUT/${s%.cpp}.o" &
    pids+=($!)
done
$CLANG -O2 -g -std=c++17 -fPIC -pthread -fsanitize=$SAN -fno-omit-frame-pointer -c "$CSRC/sc_gauss_host.cpp" -o "$OUT/sc_gauss_host.o"
$CLANG -O1 -g -std=c++17 -pthread -fsanitize=$SAN -fno-omit-frame-pointer -D__HIP_PLATFORM_AMD__ -I /opt/rocm/include -I "$ROOT/include" -c "$ROOT/tests/native/abi_sanitized.cpp" -o "$OUT/abi_sanitized.o"
for p in "${pids[@]}"; do wait "$p"; done
$HIPCC --offload-arch=gfx950 -Xarch_host -fsanitize=$SAN -o "$OUT/abi_$SAN" "$OUT"/sc_quad.o "$OUT"/sc_kernels.o "$OUT"/sc_diag.o "$OUT"/sc_api.o "$OUT"/sc_serve.o "$OUT"/sc_gauss_host.o "$OUT"/abi_sanitized.o -lquadmath -lpthread
rm -f "$OUT"/*.o
