; A kernel that forms the flat address of a stack object minus 4 and lets it
; escape (stored to global memory), then walks the object through that
; pre-decremented pointer.  With the installed AMDGPU back end (gfx950, -O3) the
; escaped value is computed as
;     s_mov_b64  s[6:7], src_private_base
;     s_add_u32  s4, 0, 0x5c        ; frame offset 0x60 and -4 folded into one immediate
;     s_addc_u32 s5, s7, -1         ; high half still adds the sign extension of -4
; The low add no longer carries, so the high half is one less than the private
; aperture's: the pointer lies 4 GiB below the aperture.  The same kernel with
; the array in LDS (addrspace 3) keeps the carry (s_add_u32 0x60, -4).
; Used by the CPU tests of the tuner's code-object gate; never run on a GPU.
target triple = "amdgcn-amd-amdhsa"

define amdgpu_kernel void @k(ptr addrspace(1) %out, ptr addrspace(1) %pout, float %v) {
entry:
  %pad = alloca [24 x i32], align 16, addrspace(5)
  %a = alloca [4 x float], align 16, addrspace(5)
  %padf = addrspacecast ptr addrspace(5) %pad to ptr
  store volatile i32 7, ptr %padf, align 4
  %f = addrspacecast ptr addrspace(5) %a to ptr
  %start = getelementptr i8, ptr %f, i64 -4
  store volatile ptr %start, ptr addrspace(1) %pout, align 8
  br label %loop
loop:
  %i = phi i32 [ 0, %entry ], [ %i1, %loop ]
  %p = phi ptr [ %start, %entry ], [ %pn, %loop ]
  %pn = getelementptr i8, ptr %p, i64 4
  store volatile float %v, ptr %pn, align 4
  %i1 = add i32 %i, 1
  %c = icmp slt i32 %i1, 4
  br i1 %c, label %loop, label %exit
exit:
  %g = getelementptr i8, ptr %f, i64 8
  %r = load volatile float, ptr %g, align 4
  store float %r, ptr addrspace(1) %out, align 4
  ret void
}
