#!/bin/bash
# Host-code sanitizer build of the library and the plain C example:
# AddressSanitizer and UndefinedBehaviorSanitizer on the host code (the C ABI,
# the FDP=H setup: tree, ART integers, ACA+, list building) and on the
# example; device code is built as usual.  Output in _build/sanitize/.
# Run the example afterwards with
#   ASAN_OPTIONS=detect_leaks=0:protect_shadow_gap=0 \
#   LD_LIBRARY_PATH=$(dirname $ASAN_RT) _build/sanitize/example N M [mode]
# (the HIP runtime maps device apertures where the shadow gap would be).
set -euo pipefail
ROOT=$(cd "$(dirname "$0")/../.." && pwd)
OUT=$ROOT/_build/sanitize
CSRC=$ROOT/paper_1903_02118_amd/csrc
HIPCC=/opt/rocm/bin/hipcc
CLANG=/opt/rocm/llvm/bin/clang
mkdir -p "$OUT"
COMMON="-O1 -g -std=c++17 -fPIC -I$ROOT/include -I$CSRC -fno-omit-frame-pointer"
DEV="-x hip --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops -munsafe-fp-atomics"
HOSTF="-x c++ -D__HIP_PLATFORM_AMD__ -I/opt/rocm/include -fopenmp"
$HIPCC $COMMON $DEV -c "$CSRC/kernels.hip" -o "$OUT/kernels.o"
$HIPCC $COMMON $DEV -c "$CSRC/probe.hip" -o "$OUT/probe.o"
$HIPCC $COMMON $HOSTF -Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined -c "$CSRC/api.cpp" -o "$OUT/api.o"
$HIPCC $COMMON $HOSTF -Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined -c "$CSRC/fdph_setup.cpp" -o "$OUT/fdph_setup.o"
$HIPCC --offload-arch=gfx950 -shared -fopenmp -Xarch_host -shared-libasan -Xarch_host -fsanitize=address \
    -Xarch_host -fsanitize=undefined -o "$OUT/libbie.so" "$OUT/kernels.o" "$OUT/probe.o" "$OUT/api.o" "$OUT/fdph_setup.o"
$CLANG -O1 -g -shared-libasan -fsanitize=address,undefined -D__HIP_PLATFORM_AMD__ -I"$ROOT/include" -I/opt/rocm/include \
    "$ROOT/tests/c_abi/example.c" -o "$OUT/example" -L"$OUT" -lbie -L/opt/rocm/lib -lamdhip64 -lm \
    -Wl,-rpath,"$OUT":/opt/rocm/lib
echo "$OUT/example"
