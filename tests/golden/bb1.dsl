fun f0(ipt: W ^ 4) -> W ^ 1 {
   opt[0] = 4;
   whl opt[0] {
      opt[0] = opt[0] + opt[0];
      scr[3] = opt[0];
      whl opt[0] {
         whl opt[0] {
            scr[7] = scr[2] * 7;
            opt[0] = 0;
            scr[1] = 9
         }
      };
      opt[0] = scr[2] + 0;
      opt[0] = scr[3] + scr[5]
   }
}
